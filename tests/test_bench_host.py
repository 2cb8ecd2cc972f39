"""Host-side checks of the benchmark script (no GPU).

The benchmark embeds rocprofv3 byte counts of the quadrature kernels together
with a SHA-256 of the kernel sources they were measured on, and reports them
as null once the sources differ.  These tests keep the committed counts tied
to the committed kernels, pin the per-unit work figures its rooflines divide
by, and check that a request for several GPUs is refused with a message.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_counts_belong_to_the_committed_kernel_sources():
    # an edit to a quadrature kernel source must come with counters taken on it
    assert bench._sources_match()
    kernels = ["pad_volume_kernel", "pad_volume_yfast_kernel", "project_kernel"]
    assert bench.measured_traffic(kernels, 3, "cone_256") > 0
    assert bench.measured_traffic(kernels, 3, "cone_512") is None  # measured on cone_256 only
    assert bench.measured_traffic(["backproject_cells_kernel"], 2, "cone_256") is None


def test_traffic_tables_cover_both_benchmarked_degrees():
    for n in (3, 0):
        for k in ("pad_volume_kernel", "project_kernel", "backproject_cells_kernel", "cells_to_coeffs_kernel"):
            r, w = bench.TRAFFIC_BYTES[(k, n)]
            assert r > 0 and w > 0
            assert bench.L2_FILL_BYTES[(k, n)] > 0


def test_unit_work_figures():
    # cubic forward per (line, knot cell), 5 Gauss-Legendre nodes of: node map
    # 3 FMA (6), three axes of blending weights (3 x 15), the 64 + 16 + 4 FMA
    # contraction (168), the weighted sum (2); plus the cell's accumulation (2)
    assert bench.fwd_unit_flops(3) == 5 * (6 + 45 + 168 + 2) + 2 == 1107
    assert bench.adj_unit_flops(3) == 722
    # degree 0: one product per (line, cell)
    assert bench.fwd_unit_flops(0) == bench.adj_unit_flops(0) == 2.0
    # per cell, the moments-to-bases map: three 4 x 4 matrices on 64 values
    assert bench.adj_cell_flops(3) == 3 * 2 * 4 ** 4
    # the network's per-pair matrix work: three 64 x 64 hidden layers, the
    # 5 -> 64 input layer and the 64 -> 1 output layer
    assert bench.MLP_FLOPS_PER_PAIR == 24576 + 640 + 128


def test_several_gpus_are_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
