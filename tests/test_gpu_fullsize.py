"""Parity at the full workload sizes, in the launch configuration the
benchmark times (one call over all views), on sampled outputs the FP64 oracle
computes one by one: 16,384 lines (seed 7) and 4,096 coefficients (seed 8).

parallel_128: 128^3, ellipsoids + noise, 240 parallel views, 192^2 detector.
cone_256:     256^3, ellipsoids, 360 cone views, 384^2 detector.
cone_512:     512^3 smooth field, one batch of 32 of its 720 cone views.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2511_11078_amd import configs, synth
from paper_2511_11078_amd.ops import Context, default_weights

from gpu_helpers import rel_l2, say, to_gpu, to_np

pytestmark = pytest.mark.gpu

TOL_QUAD = 1e-5
TOL_MLP = 1e-3
_VOLUMES = {}


def _volume(wl):
    if wl.name not in _VOLUMES:
        _VOLUMES[wl.name] = wl.volume()
    return _VOLUMES[wl.name]


def _check(wl_name, form, n_rays=16384, n_coefs=4096, views=None, noise_adjoint=False):
    """Forward on the workload's volume, and the adjoint of its own forward
    projection (and, with noise_adjoint, also of a Gaussian noise sinogram,
    seed 9, whose back-projection does not average per-pair errors away)."""
    wl = configs.get(wl_name)
    geom = wl.geometry() if views is None else wl.geometry().subset_views(*views)
    dims = wl.dims
    c_np = _volume(wl)
    ctx = Context(wl.degree, form, 0)
    c = to_gpu(c_np)
    y = ctx.project(c, geom)
    b = ctx.backproject(y, geom, dims)
    torch.cuda.synchronize()
    rays = synth.sample_indices(geom.n_rays, n_rays, seed=7)
    coefs = synth.sample_indices(int(np.prod(dims)), n_coefs, seed=8)
    y_np = to_np(y)
    ef = rel_l2(y_np.ravel()[rays], oracle.project(c_np, geom, wl.degree, rays=rays))
    eb = rel_l2(to_np(b).ravel()[coefs], oracle.backproject_subset(y_np, geom, dims, wl.degree, coefs=coefs))
    msg = f"  {wl_name} {form}: forward rel-L2 {ef:.3e}, adjoint rel-L2 {eb:.3e}"
    ebn = None
    if noise_adjoint:
        rng = np.random.default_rng(9)
        yn = rng.standard_normal(y_np.shape).astype(np.float32)
        bn = ctx.backproject(to_gpu(yn), geom, dims)
        torch.cuda.synchronize()
        ebn = rel_l2(to_np(bn).ravel()[coefs], oracle.backproject_subset(yn, geom, dims, wl.degree, coefs=coefs))
        msg += f", adjoint of noise rel-L2 {ebn:.3e}"
    say(msg)
    ctx.close()
    return (ef, eb) if not noise_adjoint else (ef, eb, ebn)


def test_parallel_128_quad():
    say("parallel_128 quad")
    ef, eb = _check("parallel_128", "quad")
    assert ef <= TOL_QUAD and eb <= TOL_QUAD


def _dot_test(wl_name, seed):
    """<A x, y> = <x, A^T y> for noise x and y over the whole workload (the
    adjoint is the exact transpose, so only FP32 rounding separates them)."""
    wl = configs.get(wl_name)
    geom = wl.geometry()
    ctx = Context(wl.degree, "quad", 0)
    rng = np.random.default_rng(seed)
    x = to_gpu(rng.standard_normal(wl.dims[::-1]).astype(np.float32))
    y = to_gpu(rng.standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32))
    Ax = ctx.project(x, geom)
    Aty = ctx.backproject(y, geom, wl.dims)
    lhs = float((Ax.double() * y.double()).sum())
    rhs = float((x.double() * Aty.double()).sum())
    rel = abs(lhs - rhs) / (float(Ax.double().norm()) * float(y.double().norm()))
    say(f"  {wl_name} dot-test relative mismatch {rel:.3e}")
    ctx.close()
    return rel


def test_parallel_128_dot_test():
    say("parallel_128 dot test")
    assert _dot_test("parallel_128", 5) <= 1e-5


def test_cone_256_dot_test():
    say("cone_256 dot test")
    assert _dot_test("cone_256", 6) <= 1e-5


def test_cone_256_quad():
    say("cone_256 quad")
    ef, eb = _check("cone_256", "quad", n_coefs=1024)
    assert ef <= TOL_QUAD and eb <= TOL_QUAD


@pytest.mark.skipif(not os.path.exists(default_weights(3)), reason="no trained network weights")
def test_parallel_128_mlp():
    say("parallel_128 mlp")
    ef, eb = _check("parallel_128", "mlp", n_coefs=1024)
    assert ef <= TOL_MLP and eb <= TOL_MLP


@pytest.mark.skipif(not os.path.exists(default_weights(3)), reason="no trained network weights")
def test_cone_256_mlp():
    """The benchmark workload with the network form, in the launch the
    benchmark times (all 360 views in one call): 16,384 sampled lines and
    1,024 sampled coefficients, the adjoint of the forward projection and of
    a noise sinogram."""
    say("cone_256 mlp")
    ef, eb, ebn = _check("cone_256", "mlp", n_coefs=1024, noise_adjoint=True)
    assert ef <= TOL_MLP and eb <= TOL_MLP and ebn <= TOL_MLP


@pytest.mark.skipif(not os.path.exists(default_weights(3)), reason="no trained network weights")
def test_cone_512_one_batch_mlp():
    say("cone_512, views 0..31, mlp")
    ef, eb = _check("cone_512", "mlp", n_rays=4096, n_coefs=256, views=(0, 32))
    assert ef <= TOL_MLP and eb <= TOL_MLP


def test_cone_512_one_batch_quad():
    say("cone_512, views 32..63, quad")
    ef, eb = _check("cone_512", "quad", n_rays=4096, n_coefs=256, views=(32, 64))
    assert ef <= 3e-5 and eb <= 3e-5
