"""GPU checks of the network form for the quadratic basis (degree 2, the
paper's own basis, Sec. 2.2) and the linear basis (degree 1), each with its
own trained weights.

The same two questions as for the cubic network: does the kernel compute the
network the blob defines on exactly the pairs of the quadrature form
(footprints against a numpy evaluation of the blob in the kernel's
arithmetic, the exact gate, the dot-product test), and how far is the
network form from the exact transform (FP64 oracle), in both directions?
The bound on the latter is the network form's stated 1e-3 for degree 2.
The degree-1 footprint has creases (beta^1 is only continuous), which a
smooth SiLU network of this size fits less well: its validation fit is
5.3e-4 on the training distribution of directions, and on the 32 spherical
Fibonacci directions of the parallel test the projections differ from the
oracle by 1.0e-3 (forward) and 1.3e-3 (adjoint of noise); its bound is
2e-3.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2511_11078_amd import footprint_net as fn
from paper_2511_11078_amd import synth
from paper_2511_11078_amd.ops import Context, default_weights

from gpu_helpers import rel_l2, say, to_gpu, to_np

pytestmark = pytest.mark.gpu

TOL_MLP = {2: 1e-3, 1: 2e-3}


@pytest.fixture(scope="module", params=[2, 1])
def deg(request):
    n = request.param
    if not os.path.exists(default_weights(n)):
        pytest.skip(f"no degree-{n} network weights")
    with open(default_weights(n), "rb") as fh:
        blob = fn.parse_blob(fh.read())
    ctx = Context(n, "mlp", 0)
    yield n, ctx, blob
    ctx.close()


def test_blob_matches_degree(deg):
    n, _, blob = deg
    assert blob["degree"] == n


def test_network_footprint_matches_numpy(deg):
    n, mctx, blob = deg
    say(f"degree-{n} network footprint vs numpy evaluation of the blob")
    rng = np.random.default_rng(400 + n)
    from paper_2511_11078_amd.train_footprint import sample_pairs
    w, x = sample_pairs(n, 30000, rng)
    w32, x32 = w.astype(np.float32), x.astype(np.float32)
    got = to_np(mctx.footprint(to_gpu(w32), to_gpu(x32)))
    wd = w32.astype(np.float64)
    wd /= np.linalg.norm(wd, axis=1, keepdims=True)
    want = fn.blob_forward(blob, fn.fold_features(wd, x32.astype(np.float64)).astype(np.float32))
    e = rel_l2(got, want)
    say(f"  rel-L2 {e:.3e}")
    assert e <= 2e-5


def test_network_gate_is_exact(deg):
    n, mctx, _ = deg
    say(f"degree-{n} network gate")
    rng = np.random.default_rng(401 + n)
    w = rng.standard_normal((5000, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    h = 0.5 * (n + 1)
    x = rng.uniform(-1.8 * h, 1.8 * h, (5000, 3))
    inside = fn.chord_nonempty(n, w, x)
    got = to_np(mctx.footprint(to_gpu(w.astype(np.float32)), to_gpu(x.astype(np.float32))))
    far = ~fn.chord_nonempty(n, w, x * 1.0005) & ~inside
    assert np.all(got[far] == 0.0)
    assert np.count_nonzero(got[inside]) > 0.95 * inside.sum()


def test_network_dot_product_test(deg):
    n, mctx, _ = deg
    say(f"degree-{n} network dot test (cone)")
    dims = (30, 27, 25)
    rng = np.random.default_rng(420 + n)
    geom = synth.cone_circular_geometry(5, 39, 43, src_radius=75.0, src_det=110.0, angle0=0.3)
    x = to_gpu(rng.standard_normal(dims[::-1]).astype(np.float32))
    y = to_gpu(rng.standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32))
    Ax = mctx.project(x, geom)
    Aty = mctx.backproject(y, geom, dims)
    lhs = float((Ax.double() * y.double()).sum())
    rhs = float((x.double() * Aty.double()).sum())
    rel = abs(lhs - rhs) / (float(Ax.double().norm()) * float(y.double().norm()))
    say(f"  dot-test relative mismatch {rel:.3e}")
    assert rel <= 1e-5


@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_network_vs_oracle(deg, kind):
    n, mctx, blob = deg
    say(f"degree-{n} network vs oracle ({kind})")
    dims = (32, 32, 32)
    c = synth.ellipsoid_phantom(dims, 6, seed=0)
    if kind == "parallel":
        geom = synth.parallel_geometry(synth.fibonacci_directions(32), 48, 48)
    else:
        geom = synth.cone_circular_geometry(24, 40, 44, src_radius=80.0, src_det=96.0, angle0=0.1)
    got = to_np(mctx.project(to_gpu(c), geom))
    want = oracle.project(c, geom, n)
    e = rel_l2(got, want)
    rng = np.random.default_rng(430 + n)
    y = rng.standard_normal(want.shape).astype(np.float32)
    coefs = synth.sample_indices(int(np.prod(dims)), 2048, seed=431)
    gb = to_np(mctx.backproject(to_gpu(y), geom, dims)).ravel()[coefs]
    wb = oracle.backproject_subset(y, geom, dims, n, coefs=coefs)
    eb = rel_l2(gb, wb)
    say(f"  forward rel-L2 {e:.3e}, adjoint (noise sinogram) rel-L2 {eb:.3e} (blob fit fp32 "
        f"{blob['rel_fp32']:.2e}, kernel arithmetic {blob['rel_bf16']:.2e})")
    assert e <= TOL_MLP[n] and eb <= TOL_MLP[n]
