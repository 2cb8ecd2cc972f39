"""Differentiation and the least-squares loop on the GPU (quadrature form).

* finite differences: L(c) = 1/2 ||A c - y||^2 is quadratic, so the central
  difference along any direction d equals <A^T(A c - y), d> up to FP32
  rounding; checked on 64 random directions through the autograd Function.
* CGLS (FP32 vectors, FP64 device scalars) against the FP64 oracle's CGLS
  driven by the oracle's own forward/adjoint, iterate by iterate, on a
  small problem; and a monotone residual on a larger one.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_11078_amd import synth
from paper_2511_11078_amd.ops import Context, Project, Projector, cgls

from gpu_helpers import rel_l2, say, tilted_parallel, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx3():
    return Context(3, "quad", 0)


def test_finite_differences_64_directions(ctx3):
    say("finite differences, 64 directions")
    dims = (24, 22, 20)
    geom = synth.cone_circular_geometry(10, 31, 33, src_radius=60.0, src_det=72.0, angle0=0.2)
    P = Projector(dims, geom, context=ctx3)
    rng = np.random.default_rng(4)
    c0 = to_gpu(synth.ellipsoid_phantom(dims, 6, seed=0))
    y = to_gpu(rng.standard_normal(P.sino_shape).astype(np.float32))

    def loss(c):
        r = (P.forward(c) - y).double()
        return 0.5 * float((r * r).sum())

    c = c0.clone().requires_grad_(True)
    r = Project.apply(c, P) - y
    (0.5 * (r * r).sum()).backward()
    g = c.grad.double()
    worst = 0.0
    for k in range(64):
        d = to_gpu(rng.standard_normal(P.vol_shape).astype(np.float32))
        Ad = P.forward(d)
        res = P.forward(c0) - y
        eps = 0.1 * float(res.double().norm()) / float(Ad.double().norm())
        fd = (loss(c0 + eps * d) - loss(c0 - eps * d)) / (2 * eps)
        an = float((g * d.double()).sum())
        err = abs(fd - an) / max(abs(an), 1e-30)
        worst = max(worst, err)
    say(f"  worst relative FD error over 64 directions: {worst:.3e}")
    assert worst <= 1e-3


def test_cgls_matches_oracle_cgls():
    say("CGLS vs oracle CGLS")
    dims = (12, 11, 10)
    geom = tilted_parallel(16, 17, 17, seed=9)
    P = Projector(dims, geom, degree=3, form="quad")
    c_true = synth.ellipsoid_phantom(dims, 6, seed=0)
    y = oracle.project(c_true, geom, 3).astype(np.float32)
    iters = 8
    x_gpu, hist = cgls(P, to_gpu(y), iters=iters)
    torch.cuda.synchronize()

    def A(v):
        return oracle.project(v.reshape(dims[::-1]).astype(np.float32), geom, 3).ravel()

    def At(r):
        return oracle.backproject_subset(r.reshape(geom.n_views, 17, 17).astype(np.float32), geom, dims,
                                         3).ravel()

    x_or, hist_or = oracle.cgls(A, At, y.ravel().astype(np.float64), iters)
    e = rel_l2(to_np(x_gpu).ravel(), x_or)
    say(f"  x rel-L2 after {iters} iterations: {e:.3e}")
    g_gpu = to_np(hist)
    g_or = np.array([h[1] ** 2 for h in hist_or])
    say(f"  ||A^T r||^2: gpu {g_gpu[-1]:.4e} oracle {g_or[-1]:.4e}")
    # the oracle's iteration rounds A c_true's FP32 rounding differently;
    # early iterates agree to FP32-level relative error
    assert e <= 1e-3
    np.testing.assert_allclose(g_gpu[:4], g_or[:4], rtol=1e-3)


def test_cgls_residual_decreases_cone():
    say("CGLS cone residual")
    dims = (40, 40, 40)
    geom = synth.cone_circular_geometry(60, 48, 48, src_radius=100.0, src_det=120.0)
    P = Projector(dims, geom, degree=3, form="quad")
    c_true = to_gpu(synth.ellipsoid_phantom(dims, 6, seed=0))
    y = P.forward(c_true)
    res = []

    def cb(k, x, r):
        res.append(float(r.double().norm()))

    x, hist = cgls(P, y, iters=20, callback=cb)
    say(f"  residual {res[0]:.3e} -> {res[-1]:.3e}")
    assert all(res[k + 1] <= res[k] * (1 + 1e-6) for k in range(len(res) - 1))
    assert res[-1] < 0.05 * float(y.double().norm())
