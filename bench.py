#!/usr/bin/env python3
"""Benchmark: forward + adjoint throughput of the spline x-ray transform.

Workload cone_256: 256^3 cubic B-spline coefficients (six random ellipsoids,
seed 0), circular cone beam of 360 views (source radius 640, source-detector
distance 768), 384 x 384 detector -- 53,084,160 lines.  One step is one
forward projection and one back-projection over all views with the chosen
footprint form (default: exact quadrature, FP32).  Inputs are resident on
the GPU before timing starts; the geometry is uploaded once beforehand.

Printed: one JSON line with rays/s = lines / (t_forward + t_adjoint), the
roofline of the dominant kernel (algorithmic work from the oracle's cell,
pair and segment counts on a 4,096-line sample, divided by the kernel's mean
duration measured with HIP events on its stream), the relative L2 error
against the FP64 oracle on 262,144 sampled lines (seed 7) and 32,768 sampled
coefficients (seed 8), and the oracle itself timed on the host as the CPU
baseline (all host threads, and one).

    python bench.py [--steps K] [--warmup W] [--form quad|mlp|pair] [--one-form]
                    [--workload NAME] [--degree N] [--views K]

By default one extra, separately timed step of each other footprint form
reports the speed-ups and errors: the network form (when its weights are
present) and the per-pair exact quadrature form, which evaluates the exact
footprint of every (line, basis) pair on the network form's traversal, so
that network vs exact footprint is compared on the same walk.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "forward+adjoint rays/s at 256³ cone-beam (MLP vs quadrature footprint), rel-L2"
# MI355X published peaks
PEAK_FP32_VECTOR_TFLOPS = 157.3      # 256 CU x 128 FP32 FMA/clk (packed) x 2 x 2.4 GHz
PEAK_BF16_MFMA_TFLOPS = 2500.0
# exp and reciprocal results per second: measured on the box by peaks_probe.hip
# (interleaved v_exp_f32 / v_rcp_f32 streams), and the quarter-rate figure
# 256 CU x 4 SIMD x 16 lanes / 4 x 2.4 GHz
PEAK_TRANS_MEASURED = 13.1
PEAK_TRANS_QUARTER_RATE = 256 * 4 * 16 / 4 * 2.4e9 / 1e12
GL_ORDER = {0: 1, 1: 2, 2: 4, 3: 5}
FORM_DTYPE = {"quad": "f32", "pair": "f32", "mlp": "bf16"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


N_SAMPLE_LINES = 262144   # parity and CPU-baseline samples (about 10 s of oracle work)
N_SAMPLE_COEFS = 32768
MLP_FLOPS_PER_PAIR = 2.0 * 3 * 64 * 64 + 2.0 * 5 * 64 + 2.0 * 64   # hidden BF16 + layer 1 + output
MLP_TRANS_PER_PAIR = 2 * 4 * 64   # SiLU of 4 x 64 hidden units: one exp and one reciprocal each


# HBM bytes per application (forward or adjoint: the launches of each kernel
# summed; the cubic forward launches project_kernel twice, once per copy of
# the coefficients) of the quadrature kernels on cone_256, from rocprofv3
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what the same
# counters read for a plain 256 MiB device copy (x2.000 and x1.000); see
# profiles/cone256_traffic_counters.md.  Valid only for the kernel sources they
# were measured on (SHA-256 over QUAD_SOURCES); otherwise reported as null.
QUAD_SOURCES = ["csrc/ss_kernels.hip", "csrc/ss_math.hpp", "csrc/ss_traverse.hpp", "csrc/ss_kernels.hpp"]
TRAFFIC_SHA256 = "369c6360167dcf2aa49bd385ba21713a13c9bf62f635122478f66696ae4d78ea"
TRAFFIC_BYTES = {  # (kernel, degree) -> (read bytes, written bytes) per application, cone_256
    ("pad_volume_kernel", 3): (2.0 * 36897 * 1024, 1.0 * 71874 * 1024),
    ("pad_volume_yfast_kernel", 3): (2.0 * 65553 * 1024, 1.0 * 72218 * 1024),
    ("project_kernel", 3): (2.0 * (1295830 + 1045866) * 1024, 1.0 * (147137 + 94671) * 1024),  # two launches
    ("backproject_cells_kernel", 3): (2.0 * 3007007 * 1024, 1.0 * 5412897 * 1024),
    ("cells_to_coeffs_kernel", 3): (2.0 * 2481303 * 1024, 1.0 * 65536 * 1024),
    ("pad_volume_kernel", 0): (2.0 * 36895 * 1024, 1.0 * 67084 * 1024),
    ("project_kernel", 0): (2.0 * 1069235 * 1024, 1.0 * 254618 * 1024),
    ("backproject_cells_kernel", 0): (2.0 * 1260068 * 1024, 1.0 * 67106 * 1024),
    ("cells_to_coeffs_kernel", 0): (2.0 * 32785 * 1024, 1.0 * 65536 * 1024),
}


# L2 -> L1 fill bytes per application on cone_256: rocprofv3 TCP_TCC_READ_REQ_sum
# times 128 bytes, the request size a plain device copy shows (1 GiB read in
# 8,388,608 requests); same source check as the HBM bytes.  The L2 peak is
# derived from the unit counts: 8 XCDs x 16 channels x 128 bytes per clock
# at 2.4 GHz; the best L2-read rate measured by peaks_probe.hip is below it.
L2_FILL_BYTES = {  # (kernel, degree) -> bytes per application, cone_256
    ("pad_volume_kernel", 3): 128.0 * 589824,
    ("pad_volume_yfast_kernel", 3): 128.0 * 1048576,
    ("project_kernel", 3): 128.0 * (12960493046 + 6705862807),  # two launches
    ("backproject_cells_kernel", 3): 128.0 * 210638300,
    ("cells_to_coeffs_kernel", 3): 128.0 * 45215857,
    ("pad_volume_kernel", 0): 128.0 * 589824,
    ("project_kernel", 0): 128.0 * 5704423358,
    ("backproject_cells_kernel", 0): 128.0 * 194942051,
    ("cells_to_coeffs_kernel", 0): 128.0 * 524288,
}
PEAK_L2_TBS = 8 * 16 * 128 * 2.4e9 / 1e12
MEASURED_L2_READ_TBS = 28.9


def _sources_match() -> bool:
    import hashlib

    h = hashlib.sha256()
    for f in QUAD_SOURCES:
        with open(os.path.join(ROOT, "paper_2511_11078_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest() == TRAFFIC_SHA256


def measured_traffic(kernels, degree: int, workload: str):
    """HBM bytes of one application (forward or adjoint) of the named kernels
    (summed), or None when they were not measured for this workload and these
    sources."""
    if workload != "cone_256" or any((k, degree) not in TRAFFIC_BYTES for k in kernels):
        return None
    if not _sources_match():
        return None
    return float(sum(sum(TRAFFIC_BYTES[(k, degree)]) for k in kernels))


def measured_l2(kernels, degree: int, workload: str, ms: float):
    """L2 -> L1 fill rate of one application of the named kernels against the
    L2 peak, or None when not measured for this workload and these sources."""
    if workload != "cone_256" or any((k, degree) not in L2_FILL_BYTES for k in kernels):
        return None
    if not _sources_match():
        return None
    b = float(sum(L2_FILL_BYTES[(k, degree)] for k in kernels))
    ach = b / (ms / 1e3) / 1e12
    return {"bytes": b, "achieved": ach, "peak": PEAK_L2_TBS, "unit": "TB/s", "frac": ach / PEAK_L2_TBS,
            "frac_of_measured_l2_read": ach / MEASURED_L2_READ_TBS}


# FP32 flops of the blending weights of one axis at one node (cell_weights):
# FMA = 2 flops, add or multiply = 1
BLEND_FLOPS = {0: 0, 1: 1, 2: 7, 3: 15}


def fwd_unit_flops(n: int) -> float:
    """Algorithmic FP32 work of one (line, knot cell) unit of the forward: at
    each of the m Gauss-Legendre nodes, the node map (3 FMA), the n+1 blending
    weights of three axes, the contraction of the (n+1)^3 coefficient block
    ((n+1)^3 + (n+1)^2 + (n+1) FMA) and the weighted sum (1 FMA), plus the
    cell's accumulation (1 FMA).  Degree 0: coefficient times chord (1 FMA)."""
    if n == 0:
        return 2.0
    nb, m = n + 1, GL_ORDER[n]
    return m * (6 + 3 * BLEND_FLOPS[n] + 2 * (nb ** 3 + nb ** 2 + nb) + 2) + 2


def adj_unit_flops(n: int) -> float:
    """Algorithmic FP32 work of one (line, knot cell) unit of the adjoint, which
    accumulates centred moments: the chord through the cell (about 32 flops:
    slab test, midpoint, half-length, centred start and step) and at each node
    the node map (3 FMA), the powers of the three coordinates ((n+1) + 2(n-1)
    multiplies, the first carrying the quadrature weight), the products of two
    axes (n(n+1) multiplies) and the accumulation ((n+1)^2 adds and n(n+1)^2
    FMA).  This is the association with the fewest flops; the kernel forms
    the n^2 products of the second and third axes instead and accumulates
    with (n+1)((n+1)^2 - 1) FMA (767 flops per unit at degree 3, in fewer
    instructions), so the figure is conservative.  Degree 0: sinogram value
    times chord (1 FMA)."""
    if n == 0:
        return 2.0
    nb, m = n + 1, GL_ORDER[n]
    node = 6 + (nb + 2 * (n - 1)) + n * nb + nb * nb + 2 * n * nb * nb
    return m * node + 32


def pair_flops(n: int, segs_per_pair: float) -> float:
    """Per-pair work of the exact footprint as counted per (line, basis) pair:
    on each of its pieces, m Gauss-Legendre nodes of (3n + 4) FMA-class
    operations (three Horner pieces of degree n, two products, the weighted
    sum, the node map), plus about 60 for the chord and the knot crossings.
    The transform's kernels do not execute this count: they share the
    nodes of one knot cell among its (n+1)^3 bases."""
    if n == 0:
        return 8.0
    return segs_per_pair * GL_ORDER[n] * (3 * n + 4) * 2.0 + 60.0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def adj_cell_flops(n: int) -> float:
    """Once per knot cell and application: the blending map from moments to
    per-basis integrals, one (n+1) x (n+1) matrix per axis on (n+1)^3 values."""
    nb = n + 1
    return 0.0 if n == 0 else 3.0 * 2 * nb ** 4


def time_form(ctx, c, geom, dims, y, b, steps, warm, form, stream):
    """Warm-up, then `steps` timed forward + adjoint steps with HIP events on
    the launch stream; returns per-step forward and adjoint times (ms)."""
    import torch

    for k in range(warm):
        ctx.project(c, geom, y)
        ctx.backproject(y, geom, dims, b)
        torch.cuda.synchronize()
        log(f"[bench] {form}: warm-up step {k + 1}/{warm} done")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for k in range(steps):
        e0, e1, e2 = ev[k]
        e0.record(stream)
        ctx.project(c, geom, y)
        e1.record(stream)
        ctx.backproject(y, geom, dims, b)
        e2.record(stream)
        e2.synchronize()
        log(f"[bench] {form}: step {k + 1}/{steps}: forward {e0.elapsed_time(e1):.1f} ms, "
            f"adjoint {e1.elapsed_time(e2):.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    tf = [e0.elapsed_time(e1) for e0, e1, _ in ev]
    ta = [e1.elapsed_time(e2) for _, e1, e2 in ev]
    return float(np.mean(tf)), float(np.mean(ta)), wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", choices=["quad", "mlp", "pair"], default="quad",
                    help="footprint form of the timed steps")
    ap.add_argument("--one-form", action="store_true",
                    help="skip the one extra step of each other footprint form (speed-up report)")
    ap.add_argument("--workload", default="cone_256")
    ap.add_argument("--degree", type=int, default=None,
                    help="override the workload's B-spline degree (0 = voxel basis, 2 = quadratic)")
    ap.add_argument("--views", type=int, default=0,
                    help="time only the first K views (one view batch of the 512^3 workload: 32)")
    ap.add_argument("--no-oracle", action="store_true", help="skip parity and CPU baseline (profiling runs)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py measures one GPU only: the library runs the transform on a single MI355X; "
              f"--gpus {args.gpus} is not supported (views would be sharded across GPUs with an all-reduce "
              f"of the back-projected volume, which the library does not implement).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2511_11078_amd import configs, synth
    from paper_2511_11078_amd.ops import Context, default_weights

    wl = configs.get(args.workload)
    dims = wl.dims
    n = wl.degree if args.degree is None else args.degree
    geom = wl.geometry()
    if args.views:
        geom = geom.subset_views(0, min(args.views, geom.n_views))
    R = geom.n_rays
    dev = torch.device("cuda", 0)
    log(f"[bench] workload {wl.name}: dims {dims}, {geom.n_views} views, detector "
        f"{geom.det_rows}x{geom.det_cols}, {R} lines, degree {n}")
    t0 = time.time()
    c_np = wl.volume()
    log(f"[bench] phantom built in {time.time() - t0:.1f}s")
    c = torch.from_numpy(c_np).to(dev)
    y = torch.empty((geom.n_views, geom.det_rows, geom.det_cols), dtype=torch.float32, device=dev)
    b = torch.empty_like(c)

    forms = [args.form]
    if not args.one_form:
        for other in ("quad", "pair", "mlp"):
            if other == args.form or (other != "quad" and n == 0):
                continue
            if other == "mlp" and not os.path.exists(default_weights(n)):
                continue
            forms.append(other)

    ys = synth.sample_indices(R, N_SAMPLE_LINES, seed=7)
    cs = synth.sample_indices(int(np.prod(dims)), N_SAMPLE_COEFS, seed=8)
    ys_t = torch.from_numpy(ys).to(dev)
    cs_t = torch.from_numpy(cs).to(dev)
    results = {}
    y_main = None
    for fi, form in enumerate(forms):
        ctx = Context(n, form, 0)
        stream = torch.cuda.current_stream(dev)
        steps = args.steps if fi == 0 else 1
        warm = args.warmup if fi == 0 else 0
        if fi > 0:
            # an untimed first call of the extra form (its context's scratch
            # is allocated on first use), then its single timed step
            ctx.project(c, geom, y)
            ctx.backproject(y, geom, dims, b)
            torch.cuda.synchronize()
        fwd_ms, adj_ms, wall = time_form(ctx, c, geom, dims, y, b, steps, warm, form, stream)
        if fi == 0:
            y_main = y.clone()
        else:
            # parity samples: every form's adjoint is applied to the main form's sinogram
            ctx.backproject(y_main, geom, dims, b)
        torch.cuda.synchronize()
        results[form] = {"fwd_ms": fwd_ms, "adj_ms": adj_ms, "wall_s": wall, "steps": steps,
                         "y_sample": y.reshape(-1)[ys_t].cpu().numpy(),
                         "b_sample": b.reshape(-1)[cs_t].cpu().numpy()}
        ctx.close()

    main_form = forms[0]
    r0 = results[main_form]
    ms_per_step = r0["fwd_ms"] + r0["adj_ms"]
    value = R / (ms_per_step / 1e3)

    cfg = {"workload": wl.name, "dims": list(dims), "views": geom.n_views,
           "detector": [geom.det_rows, geom.det_cols], "rays": R, "geometry": geom.kind,
           "degree": n, "form": main_form}
    if args.views:
        cfg["views_of_workload"] = wl.geometry().n_views
    out = {"metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": FORM_DTYPE[main_form], "data": "synthetic", "config": cfg}

    if not args.no_oracle:
        import oracle

        y_adj_in = y_main.cpu().numpy()
        # oracle on the samples: forward lines, adjoint coefficients (same input y)
        nthreads = oracle.num_threads()
        t0 = time.perf_counter()
        yo = oracle.project(c_np, geom, n, rays=ys)
        t_of = time.perf_counter() - t0
        log(f"[bench] oracle forward on {ys.size} lines: {t_of:.1f}s")
        t0 = time.perf_counter()
        bo = oracle.backproject_subset(y_adj_in, geom, dims, n, coefs=cs)
        t_ob = time.perf_counter() - t0
        log(f"[bench] oracle adjoint on {cs.size} coefficients: {t_ob:.1f}s")
        # the same oracle on one thread, on the first 1/16 of each sample
        oracle.set_num_threads(1)
        ys1, cs1 = ys[::16], cs[::32]
        t0 = time.perf_counter()
        oracle.project(c_np, geom, n, rays=ys1)
        t1f = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.backproject_subset(y_adj_in, geom, dims, n, coefs=cs1)
        t1b = time.perf_counter() - t0
        oracle.set_num_threads(0)
        log(f"[bench] oracle on one thread: {ys1.size} lines {t1f:.1f}s, {cs1.size} coefficients {t1b:.1f}s")
        rel = {}
        for form in forms:
            rf = float(np.linalg.norm(results[form]["y_sample"] - yo) / np.linalg.norm(yo))
            ra = float(np.linalg.norm(results[form]["b_sample"] - bo) / np.linalg.norm(bo))
            rel[form] = {"forward_rel_l2": rf, "adjoint_rel_l2": ra}
        out["rel_l2_vs_oracle"] = rel[main_form]
        # algorithmic work (oracle counts on 4,096 of the sampled lines):
        # (line, basis) pairs and their footprint segments, and knot cells per line
        cnt_rays = ys[:: max(1, ys.size // 4096)][:4096]  # spread over all views (ys is sorted)
        pairs, segs = oracle.counts(dims, geom, n, rays=cnt_rays)
        cells = oracle.direct_counts(dims, geom, n, rays=cnt_rays)
        pairs_per_ray = float(pairs.mean())
        segs_per_pair = float(segs.sum() / max(pairs.sum(), 1))
        cells_per_ray = float(cells.mean())
        total_pairs = pairs_per_ray * R

        def form_kernels(form, fwd_ms, adj_ms):
            ks = []
            if form == "quad":
                nb3 = (n + 1) ** 3
                ncells = float(np.prod([d + n for d in dims]))
                fl_f = R * cells_per_ray * fwd_unit_flops(n)
                fl_a = (R * cells_per_ray * adj_unit_flops(n) + ncells * adj_cell_flops(n)
                        + nb3 * float(np.prod(dims)))
                # degree 3 walks each view in one of two copies of the
                # coefficients (x or y fastest): two pads, two launches
                fwd_name = (f"pad_volume_kernel + pad_volume_yfast_kernel + project_kernel<{n}> "
                            f"(knot-cell walk, two launches)" if n == 3 else
                            f"pad_volume_kernel + project_kernel<{n}> (knot-cell walk)")
                for name, ms, fl, unit in (
                        (fwd_name, fwd_ms, fl_f,
                         f"{fwd_unit_flops(n):.0f} flop per (line, cell) x {cells_per_ray:.1f} cells/line"),
                        (f"backproject_cells_kernel<{n}> + cells_to_coeffs_kernel<{n}> (knot-cell gather)",
                         adj_ms, fl_a,
                         f"{adj_unit_flops(n):.0f} flop per (line, cell) x {cells_per_ray:.1f} cells/line + "
                         f"{adj_cell_flops(n):.0f} per cell + {nb3} per coefficient")):
                    ach = fl / (ms / 1e3) / 1e12
                    knames = [part.strip().split("<")[0] for part in name.split(" (")[0].split("+")]
                    pp = total_pairs * pair_flops(n, segs_per_pair) / (ms / 1e3) / 1e12
                    entry = {"kernel": name, "ms": ms, "bound": "alu", "achieved": ach,
                             "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                             "frac": ach / PEAK_FP32_VECTOR_TFLOPS, "work": unit}
                    l2 = measured_l2(knames, n, wl.name, ms)
                    if l2 is not None and l2["frac"] > entry["frac"]:
                        # the cheap footprint leaves the walk bound by L2 -> L1 fills
                        entry["alu"] = {k: entry[k] for k in ("achieved", "peak", "unit", "frac", "work")}
                        entry.update(bound="l2", achieved=l2["achieved"], peak=l2["peak"], unit=l2["unit"],
                                     frac=l2["frac"], work=f"{l2['bytes'] / 1e9:.0f} GB of L2 -> L1 fills per "
                                                           f"launch (TCP_TCC_READ_REQ x 128 bytes)")
                    entry["l2"] = l2
                    entry["traffic"] = measured_traffic(knames, n, wl.name)
                    entry["per_pair_count"] = {
                        "flop_per_pair": pair_flops(n, segs_per_pair),
                        "pairs_per_line": pairs_per_ray, "achieved": pp,
                        "frac": pp / PEAK_FP32_VECTOR_TFLOPS,
                        "note": "exact footprint counted per (line, basis) pair; the kernels share "
                                "each knot cell's nodes among its bases, so this count exceeds "
                                "the work executed"}
                    ks.append(entry)
            elif form == "pair":
                fl = total_pairs * pair_flops(n, segs_per_pair)
                for name, ms in ((f"project_pair_kernel<{n}>", fwd_ms), (f"backproject_pair_kernel<{n}>", adj_ms)):
                    ach = fl / (ms / 1e3) / 1e12
                    ks.append({"kernel": name, "ms": ms, "bound": "alu", "achieved": ach,
                               "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s", "traffic": None,
                               "frac": ach / PEAK_FP32_VECTOR_TFLOPS,
                               "work": f"{pair_flops(n, segs_per_pair):.0f} flop per pair x "
                                       f"{pairs_per_ray:.0f} pairs/line"})
            else:
                trans = total_pairs * MLP_TRANS_PER_PAIR
                fl = total_pairs * MLP_FLOPS_PER_PAIR
                for name, ms in ((f"project_mlp_kernel<{n}>", fwd_ms), (f"backproject_mlp_kernel<{n}>", adj_ms)):
                    ach = trans / (ms / 1e3) / 1e12
                    mf = fl / (ms / 1e3) / 1e12
                    ks.append({"kernel": name, "ms": ms, "bound": "transcendental", "achieved": ach,
                               "peak": PEAK_TRANS_MEASURED, "unit": "T results/s", "traffic": None,
                               "frac": ach / PEAK_TRANS_MEASURED,
                               "frac_of_quarter_rate": ach / PEAK_TRANS_QUARTER_RATE,
                               "work": f"{MLP_TRANS_PER_PAIR} exp + reciprocal results per pair x "
                                       f"{pairs_per_ray:.0f} pairs/line",
                               "mfma": {"achieved": mf, "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                                        "frac": mf / PEAK_BF16_MFMA_TFLOPS,
                                        "work": f"{MLP_FLOPS_PER_PAIR:.0f} algorithmic flop per pair; the "
                                                f"kernel runs each hidden layer's product twice (two BF16 "
                                                f"terms per activation)"}})
            return ks

        kernels = form_kernels(main_form, r0["fwd_ms"], r0["adj_ms"])
        dom = max(kernels, key=lambda k: k["ms"])
        out["roofline"] = {"bound": dom["bound"], "achieved": dom["achieved"], "peak": dom["peak"],
                           "unit": dom["unit"], "frac": dom["frac"], "traffic": dom["traffic"],
                           "kernel": dom["kernel"], "kernel_ms": dom["ms"], "work": dom["work"]}
        out["kernels"] = kernels
        out["work_counts"] = {"sample_lines": int(cnt_rays.size), "pairs_per_line": pairs_per_ray,
                              "segments_per_pair": segs_per_pair, "cells_per_line": cells_per_ray,
                              "pairs_per_application": total_pairs}
        # CPU baseline: the oracle as it stands, extrapolated from its samples
        t_fwd_all = t_of * R / ys.size
        t_adj_all = t_ob * float(np.prod(dims)) / cs.size
        t1_all = t1f * R / ys1.size + t1b * float(np.prod(dims)) / cs1.size
        out["cpu_baseline"] = {"value": R / (t_fwd_all + t_adj_all), "unit": "rays/s",
                               "cores": nthreads, "kind": "oracle", "cpu_model": cpu_model(),
                               "one_thread": {"value": R / t1_all, "unit": "rays/s",
                                              "sample": f"{ys1.size} lines ({t1f:.1f}s) + {cs1.size} "
                                                        f"coefficients ({t1b:.1f}s)"},
                               "sample": f"FP64 oracle: direct line integrals of {ys.size} sampled lines "
                                         f"({t_of:.1f}s) + voxel-driven adjoint of {cs.size} sampled "
                                         f"coefficients over all {geom.n_views} views ({t_ob:.1f}s), "
                                         f"extrapolated to {R} lines and {int(np.prod(dims))} coefficients"}
        if len(forms) > 1:
            out["forms"] = {}
            for form in forms:
                rf = results[form]
                ks = form_kernels(form, rf["fwd_ms"], rf["adj_ms"])
                out["forms"][form] = {"rays_per_s": R / ((rf["fwd_ms"] + rf["adj_ms"]) / 1e3),
                                      "forward_ms": rf["fwd_ms"], "adjoint_ms": rf["adj_ms"],
                                      "forward_rel_l2": rel[form]["forward_rel_l2"],
                                      "adjoint_rel_l2": rel[form]["adjoint_rel_l2"],
                                      "roofline": [{k: kk[k] for k in ("kernel", "bound", "achieved", "peak",
                                                                       "unit", "frac")} for kk in ks]}
            q = out["forms"].get("quad")
            m = out["forms"].get("mlp")
            pq = out["forms"].get("pair")
            if q and m:
                out["forms"]["mlp_speedup_vs_quad"] = m["rays_per_s"] / q["rays_per_s"]
            if pq and m:
                # network vs exact footprint on the same walk and brick gather
                out["forms"]["mlp_speedup_vs_pair"] = m["rays_per_s"] / pq["rays_per_s"]
    out["timing"] = {"forward_ms": r0["fwd_ms"], "adjoint_ms": r0["adj_ms"], "wall_s_timed": r0["wall_s"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
