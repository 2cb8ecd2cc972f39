"""The allocation-free forward ss_project_noalloc, called through the C ABI,
against ss_project of a quadrature-form context: bit-identical sinograms
(the same kernels on the same inputs) on two calls in a row, the first at
the full cone_256 workload (the largest problem the static scratch is sized
for), the second smaller, with another geometry kind and degree, so that
the array's left-over contents of the first call must not leak into the
second."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2511_11078_amd import _lib, configs, synth
from paper_2511_11078_amd.ops import Context

from gpu_helpers import say, to_gpu

pytestmark = pytest.mark.gpu


def _noalloc(degree, c, geom, out):
    lib = _lib.load()
    g = _lib.GeometryArg(geom)
    dims = (c.shape[2], c.shape[1], c.shape[0])
    st = ctypes.c_void_p(torch.cuda.current_stream(0).cuda_stream)
    return lib.ss_project_noalloc(0, degree, ctypes.c_void_p(c.data_ptr()), _lib.dims_arg(dims), g.ref(),
                                  ctypes.c_void_p(out.data_ptr()), st)


def test_noalloc_forward_matches_project_on_two_calls():
    wl = configs.get("cone_256")
    cases = [(3, wl.volume(), wl.geometry()),
             (2, np.random.default_rng(7).standard_normal((17, 19, 23)).astype(np.float32),
              synth.parallel_geometry(synth.uniform_directions(4, seed=8), 21, 26, pitch=0.9))]
    for degree, c_np, geom in cases:
        say(f"noalloc forward: degree {degree}, dims {c_np.shape[::-1]}, {geom.kind}, {geom.n_views} views")
        c = to_gpu(c_np)
        shape = (geom.n_views, geom.det_rows, geom.det_cols)
        got = torch.full(shape, float("nan"), dtype=torch.float32, device=c.device)
        st = _noalloc(degree, c, geom, got)
        assert st == _lib.SS_OK, _lib.last_error()
        ctx = Context(degree, "quad", 0)
        want = ctx.project(c, geom)
        torch.cuda.synchronize()
        ctx.close()
        say(f"  max abs difference {float((got - want).abs().max()):.3e}")
        assert torch.equal(got, want)
