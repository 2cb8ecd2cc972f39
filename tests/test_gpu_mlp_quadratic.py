"""GPU checks of the network form for the quadratic basis (degree 2, the
paper's own basis, Sec. 2.2), with its own trained weights.

The same two questions as for the cubic network: does the kernel compute the
network the blob defines on exactly the pairs of the quadrature form, and
how far is the network form from the exact transform (FP64 oracle)?
"""
import os

import numpy as np
import pytest

import oracle
from paper_2511_11078_amd import footprint_net as fn
from paper_2511_11078_amd import synth
from paper_2511_11078_amd.ops import Context, default_weights

from gpu_helpers import rel_l2, say, tilted_parallel, to_gpu, to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not os.path.exists(default_weights(2)), reason="no degree-2 network weights")]

N = 2


@pytest.fixture(scope="module")
def mctx():
    return Context(N, "mlp", 0)


@pytest.fixture(scope="module")
def blob():
    with open(default_weights(N), "rb") as fh:
        return fn.parse_blob(fh.read())


def test_blob_is_degree_2(blob):
    assert blob["degree"] == N


def test_network_footprint_matches_numpy_quadratic(mctx, blob):
    say("degree-2 network footprint vs numpy evaluation of the blob")
    rng = np.random.default_rng(400)
    from paper_2511_11078_amd.train_footprint import sample_pairs
    w, x = sample_pairs(N, 30000, rng)
    w32, x32 = w.astype(np.float32), x.astype(np.float32)
    got = to_np(mctx.footprint(to_gpu(w32), to_gpu(x32)))
    wd = w32.astype(np.float64)
    wd /= np.linalg.norm(wd, axis=1, keepdims=True)
    want = fn.blob_forward(blob, fn.fold_features(wd, x32.astype(np.float64)).astype(np.float32))
    e = rel_l2(got, want)
    say(f"  rel-L2 {e:.3e}")
    assert e <= 2e-4


def test_network_gate_is_exact_quadratic(mctx):
    say("degree-2 network gate")
    rng = np.random.default_rng(401)
    w = rng.standard_normal((5000, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    x = rng.uniform(-3.5, 3.5, (5000, 3))
    inside = fn.chord_nonempty(N, w, x)
    got = to_np(mctx.footprint(to_gpu(w.astype(np.float32)), to_gpu(x.astype(np.float32))))
    far = ~fn.chord_nonempty(N, w, x * 1.0005) & ~inside
    assert np.all(got[far] == 0.0)
    assert np.count_nonzero(got[inside]) > 0.95 * inside.sum()


def test_network_dot_product_test_quadratic(mctx):
    say("degree-2 network dot test (cone)")
    dims = (30, 27, 25)
    rng = np.random.default_rng(420)
    geom = synth.cone_circular_geometry(5, 39, 43, src_radius=75.0, src_det=110.0, angle0=0.3)
    x = to_gpu(rng.standard_normal(dims[::-1]).astype(np.float32))
    y = to_gpu(rng.standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32))
    Ax = mctx.project(x, geom)
    Aty = mctx.backproject(y, geom, dims)
    lhs = float((Ax.double() * y.double()).sum())
    rhs = float((x.double() * Aty.double()).sum())
    rel = abs(lhs - rhs) / (float(Ax.double().norm()) * float(y.double().norm()))
    say(f"  dot-test relative mismatch {rel:.3e}")
    assert rel <= 1e-4


@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_network_vs_oracle_quadratic(mctx, blob, kind):
    say(f"degree-2 network vs oracle ({kind})")
    dims = (32, 32, 32)
    c = synth.ellipsoid_phantom(dims, 6, seed=0)
    if kind == "parallel":
        geom = synth.parallel_geometry(synth.fibonacci_directions(32), 48, 48)
    else:
        geom = synth.cone_circular_geometry(24, 40, 44, src_radius=80.0, src_det=96.0, angle0=0.1)
    got = to_np(mctx.project(to_gpu(c), geom))
    want = oracle.project(c, geom, N)
    e = rel_l2(got, want)
    rng = np.random.default_rng(430)
    y = rng.standard_normal(want.shape).astype(np.float32)
    coefs = synth.sample_indices(int(np.prod(dims)), 2048, seed=431)
    gb = to_np(mctx.backproject(to_gpu(y), geom, dims)).ravel()[coefs]
    wb = oracle.backproject_subset(y, geom, dims, N, coefs=coefs)
    eb = rel_l2(gb, wb)
    say(f"  forward rel-L2 {e:.3e}, adjoint rel-L2 {eb:.3e} (blob fit fp32 {blob['rel_fp32']:.2e}, "
        f"bf16 {blob['rel_bf16']:.2e})")
    # line sums average the per-pair fitting errors; a noise sinogram
    # back-projected does not
    assert e <= 1e-3 and eb <= 1e-2
