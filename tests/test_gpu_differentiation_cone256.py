"""Differentiation and the least-squares loop at the full cone_256 workload
(256^3 cubic coefficients, 360 cone-beam views on a circle of radius 640,
384 x 384 detector; Sec. 3, eq. (6)), quadrature form, through the autograd
Function and the device CGLS.

* finite differences on 64 random coefficient directions (seed 4):
  L(c) = 1/2 ||A c - y||^2 is quadratic, so the central difference equals
  <A^T (A c - y), d> up to FP32 rounding; each direction to 1e-3.  The
  difference L(c + e d) - L(c - e d) is formed as the inner product
  1/2 <A(c + e d) - A(c - e d), A(c + e d) + A(c - e d) - 2 y> in FP64, which
  equals it exactly and avoids subtracting two large sums;
  e = 0.1 ||A c - y|| / ||A d||.
* CGLS, 50 iterations from x = 0 on y = A c_true + Gaussian noise of variance
  1e-3 (FP32 vectors, FP64 scalars on the device): the data residual
  ||y - A x_k|| never increases, the normal-equation residual ||A^T r_k||
  falls, and the time per iteration is reported.
"""
import time

import numpy as np
import pytest
import torch

from paper_2511_11078_amd import configs
from paper_2511_11078_amd.ops import Context, Project, Projector, cgls

from gpu_helpers import say, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cone256():
    wl = configs.get("cone_256")
    geom = wl.geometry()
    ctx = Context(3, "quad", 0)
    P = Projector(wl.dims, geom, context=ctx)
    c_true = to_gpu(wl.volume())
    y_clean = P.forward(c_true).clone()
    g = torch.Generator(device=y_clean.device)
    g.manual_seed(1)
    y = y_clean + np.sqrt(1e-3) * torch.randn(y_clean.shape, generator=g, device=y_clean.device)
    yield P, c_true, y
    ctx.close()


def test_cone_256_finite_differences_64_directions(cone256):
    P, c_true, y = cone256
    say("cone_256 finite differences, 64 directions")
    c0 = 0.5 * c_true
    c = c0.clone().requires_grad_(True)
    yhat = Project.apply(c, P)
    (0.5 * ((yhat.double() - y.double()) ** 2).sum()).backward()
    grad = c.grad.double()
    res = (P.forward(c0) - y).double()
    rn = float(res.norm())
    g = torch.Generator(device=y.device)
    g.manual_seed(4)
    worst = 0.0
    t0 = time.time()
    for k in range(64):
        d = torch.randn(c0.shape, generator=g, device=y.device)
        eps = 0.1 * rn / float(P.forward(d).double().norm())
        yp = P.forward(c0 + eps * d).double()
        ym = P.forward(c0 - eps * d).double()
        dl = 0.5 * float(((yp - ym) * (yp + ym - 2.0 * y.double())).sum())
        fd = dl / (2.0 * eps)
        an = float((grad * d.double()).sum())
        err = abs(fd - an) / max(abs(an), 1e-300)
        worst = max(worst, err)
        if k % 16 == 15:
            say(f"  {k + 1} directions, worst relative error so far {worst:.3e} ({time.time() - t0:.0f}s)")
    say(f"  worst relative FD error over 64 directions: {worst:.3e}")
    assert worst <= 1e-3


def test_cone_256_cgls_50_iterations(cone256):
    P, c_true, y = cone256
    say("cone_256 CGLS, 50 iterations")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    x, hist, rhist = cgls(P, y, iters=50, residuals=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    r = torch.sqrt(rhist).cpu().numpy()
    s = torch.sqrt(hist).cpu().numpy()
    rel_x = float((x - c_true).double().norm() / c_true.double().norm())
    say(f"  {ms / 50:.1f} ms per iteration (one forward, one adjoint, three FP64 inner products, "
        f"three vector updates)")
    say(f"  ||r||: {r[0]:.4e} -> {r[10]:.4e} (10) -> {r[-1]:.4e} (50); ||A^T r||: {s[0]:.3e} -> {s[-1]:.3e}; "
        f"||x - c_true|| / ||c_true|| = {rel_x:.3e}")
    assert np.all(np.isfinite(r)) and np.all(np.isfinite(s))
    assert all(r[k + 1] <= r[k] * (1 + 1e-6) for k in range(50))
    assert r[-1] < 0.02 * r[0]
    assert s[-1] < 1e-2 * s[0]
    # the residual at the end is recomputed from the iterate
    r_direct = float((y - P.forward(x)).double().norm())
    assert abs(r_direct - r[-1]) <= 1e-3 * r[-1] + 1e-6 * r[0]
