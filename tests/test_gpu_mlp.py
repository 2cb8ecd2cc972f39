"""GPU checks of the network form (BF16 MFMA footprint).

Two separate questions:

1. Does the kernel compute the network the blob defines, on exactly the
   pairs the quadrature form visits?  Compared with a numpy evaluation of
   the same weights in the kernel's arithmetic (FP32 features and layer 1,
   BF16 hidden weights, each activation entering a hidden layer as the sum
   of two BF16 numbers, FP32 output), per footprint and per projection
   (brute-force pair enumeration on small volumes), plus the dot-product
   test of the network forward/adjoint pair.
2. How far is the network form from the exact transform?  Relative L2
   error against the FP64 oracle, in both directions (the adjoint of a
   noise sinogram, which does not average the per-pair errors away),
   bounded by the stated 1e-3 (the network's own fitting error is in the
   blob header).
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2511_11078_amd import footprint_net as fn
from paper_2511_11078_amd import synth
from paper_2511_11078_amd.ops import Context, default_weights

from gpu_helpers import rel_l2, say, tilted_parallel, to_gpu, to_np

pytestmark = pytest.mark.gpu

WEIGHTS = default_weights(3)


@pytest.fixture(scope="module")
def mctx():
    assert os.path.exists(WEIGHTS), f"trained weights missing: {WEIGHTS}"
    return Context(3, "mlp", 0)


@pytest.fixture(scope="module")
def blob():
    with open(WEIGHTS, "rb") as fh:
        return fn.parse_blob(fh.read())


def _pairs_reference(blob, n, c, geom, rays=None):
    """Brute force: every (line, coefficient) pair with a non-empty chord,
    network evaluated in numpy.  Returns the projection of c (FP64 sums)."""
    a, w = oracle.make_rays(geom, rays)
    N3, N2, N1 = c.shape
    ks = np.stack(np.meshgrid(np.arange(N1), np.arange(N2), np.arange(N3), indexing="ij"), -1).reshape(-1, 3)
    xk = ks - 0.5 * (np.array([N1, N2, N3]) - 1)
    cflat = c.transpose(2, 1, 0).reshape(-1).astype(np.float64)  # order matches ks
    out = np.zeros(a.shape[0])
    for r in range(a.shape[0]):
        x = a[r][None, :] - xk
        ww = np.broadcast_to(w[r], x.shape)
        m = fn.chord_nonempty(n, ww, x)
        if not m.any():
            continue
        f = fn.fold_features(ww[m], x[m]).astype(np.float32)
        out[r] = (fn.blob_forward(blob, f).astype(np.float64) * cflat[m]).sum()
    return out


def test_network_footprint_matches_numpy(mctx, blob):
    say("network footprint vs numpy evaluation of the blob")
    rng = np.random.default_rng(300)
    from paper_2511_11078_amd.train_footprint import sample_pairs
    w, x = sample_pairs(3, 30000, rng)
    w32, x32 = w.astype(np.float32), x.astype(np.float32)
    got = to_np(mctx.footprint(to_gpu(w32), to_gpu(x32)))
    wd = w32.astype(np.float64)
    wd /= np.linalg.norm(wd, axis=1, keepdims=True)
    want = fn.blob_forward(blob, fn.fold_features(wd, x32.astype(np.float64)).astype(np.float32))
    e = rel_l2(got, want)
    mx = np.abs(got - want).max()
    say(f"  rel-L2 {e:.3e}, max abs diff {mx:.3e}")
    # the split activations keep about 16 bits: only FP32 rounding of the
    # features, the layer-1 sums and the SiLU separates kernel and numpy
    assert e <= 2e-5 and mx <= 2e-4 * np.abs(want).max()


def test_network_gate_is_exact(mctx):
    say("network gate")
    rng = np.random.default_rng(301)
    w = rng.standard_normal((5000, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    x = rng.uniform(-4.5, 4.5, (5000, 3))
    inside = fn.chord_nonempty(3, w, x)
    got = to_np(mctx.footprint(to_gpu(w.astype(np.float32)), to_gpu(x.astype(np.float32))))
    far = ~fn.chord_nonempty(3, w, x * 1.0005) & ~inside
    assert np.all(got[far] == 0.0)
    assert np.count_nonzero(got[inside]) > 0.95 * inside.sum()


def _pairs_reference_adjoint(blob, n, y, geom, dims):
    """Brute force transpose: every (line, coefficient) pair with a
    non-empty chord adds y_line times the network value (numpy) to the
    coefficient.  Returns [N3, N2, N1] FP64 sums."""
    a, w = oracle.make_rays(geom)
    N1, N2, N3 = dims
    ks = np.stack(np.meshgrid(np.arange(N1), np.arange(N2), np.arange(N3), indexing="ij"), -1).reshape(-1, 3)
    xk = ks - 0.5 * (np.array([N1, N2, N3]) - 1)
    yf = y.reshape(-1).astype(np.float64)
    out = np.zeros(ks.shape[0])
    for r in range(a.shape[0]):
        x = a[r][None, :] - xk
        ww = np.broadcast_to(w[r], x.shape)
        m = fn.chord_nonempty(n, ww, x)
        if not m.any():
            continue
        f = fn.fold_features(ww[m], x[m]).astype(np.float32)
        out[m] += yf[r] * fn.blob_forward(blob, f).astype(np.float64)
    return out.reshape(N1, N2, N3).transpose(2, 1, 0)


@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_network_adjoint_matches_pair_enumeration(mctx, blob, kind):
    """The adjoint's waves evaluate their lanes' pairs 64 at a time and add
    each term to its owner's sum: per coefficient the same pairs and network
    values as a brute-force transpose in numpy."""
    say(f"network adjoint vs pair enumeration {kind}")
    dims = (11, 9, 7)
    rng = np.random.default_rng(315)
    if kind == "parallel":
        geom = tilted_parallel(3, 13, 15, seed=316)
    else:
        geom = synth.cone_circular_geometry(3, 14, 13, src_radius=30.0, src_det=45.0, angle0=0.25)
    y = rng.standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32)
    got = to_np(mctx.backproject(to_gpu(y), geom, dims))
    want = _pairs_reference_adjoint(blob, 3, y, geom, dims)
    e = rel_l2(got, want)
    say(f"  rel-L2 {e:.3e}")
    # the per-pair differences are those of the forward check (features
    # rounded to FP32 from differently anchored coordinates); with a noise
    # sinogram the sums cancel, so the relative error of the result is
    # larger (1.8e-5 and 1.0e-5 measured)
    assert e <= 3e-5


def test_network_deterministic(mctx):
    """Repeated calls give identical results in both directions; the
    volume spans many coefficient bricks and each wave's pair ring wraps
    many times."""
    say("network determinism")
    dims = (30, 27, 25)
    rng = np.random.default_rng(317)
    geom = synth.cone_circular_geometry(4, 39, 43, src_radius=75.0, src_det=110.0, angle0=0.3)
    x = to_gpu(rng.standard_normal(dims[::-1]).astype(np.float32))
    y = to_gpu(rng.standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32))
    f1, f2 = to_np(mctx.project(x, geom)), to_np(mctx.project(x, geom))
    b1, b2 = to_np(mctx.backproject(y, geom, dims)), to_np(mctx.backproject(y, geom, dims))
    assert np.array_equal(f1, f2)
    assert np.array_equal(b1, b2)


@pytest.mark.parametrize("kind", ["parallel", "cone", "cone_source_inside"])
def test_network_projection_matches_pair_enumeration(mctx, blob, kind):
    say(f"network projection vs pair enumeration {kind}")
    dims = (11, 9, 7)
    rng = np.random.default_rng(310)
    c = rng.uniform(0.0, 1.0, dims[::-1]).astype(np.float32)
    if kind == "parallel":
        geom = tilted_parallel(3, 13, 15, seed=311)
    elif kind == "cone":
        geom = synth.cone_circular_geometry(3, 14, 13, src_radius=30.0, src_det=45.0, angle0=0.25)
    else:  # lines through a source inside the volume (whole lines)
        geom = synth.cone_circular_geometry(3, 14, 13, src_radius=2.5, src_det=10.0, angle0=0.25)
    got = to_np(mctx.project(to_gpu(c), geom)).ravel()
    want = _pairs_reference(blob, 3, c, geom)
    e = rel_l2(got, want)
    say(f"  rel-L2 {e:.3e}")
    assert e <= 2e-5


@pytest.mark.parametrize("kind", ["parallel", "cone", "cone_source_inside"])
def test_network_dot_product_test(mctx, kind):
    say(f"network dot test {kind}")
    dims = (30, 27, 25)
    rng = np.random.default_rng(320)
    if kind == "parallel":
        geom = tilted_parallel(5, 41, 37, seed=321)
    elif kind == "cone":
        geom = synth.cone_circular_geometry(5, 39, 43, src_radius=75.0, src_det=110.0, angle0=0.3)
    else:  # coefficient boxes across the source plane take the whole detector
        geom = synth.cone_circular_geometry(3, 24, 26, src_radius=4.0, src_det=16.0, angle0=0.3)
    x = to_gpu(rng.standard_normal(dims[::-1]).astype(np.float32))
    y = to_gpu(rng.standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32))
    Ax = mctx.project(x, geom)
    Aty = mctx.backproject(y, geom, dims)
    lhs = float((Ax.double() * y.double()).sum())
    rhs = float((x.double() * Aty.double()).sum())
    rel = abs(lhs - rhs) / (float(Ax.double().norm()) * float(y.double().norm()))
    say(f"  dot-test relative mismatch {rel:.3e}")
    # forward and adjoint evaluate the same network on the same pairs; only
    # the FP32 rounding of the features differs (crossing point vs re-based
    # anchor)
    assert rel <= 1e-5


def test_network_vs_oracle_small_parallel_32(mctx, blob):
    say("network vs oracle small_parallel_32")
    dims = (32, 32, 32)
    c = synth.ellipsoid_phantom(dims, 6, seed=0)
    geom = synth.parallel_geometry(synth.fibonacci_directions(32), 48, 48)
    got = to_np(mctx.project(to_gpu(c), geom))
    want = oracle.project(c, geom, 3)
    e = rel_l2(got, want)
    rng = np.random.default_rng(330)
    y = rng.standard_normal(want.shape).astype(np.float32)
    coefs = synth.sample_indices(int(np.prod(dims)), 2048, seed=331)
    gb = to_np(mctx.backproject(to_gpu(y), geom, dims)).ravel()[coefs]
    wb = oracle.backproject_subset(y, geom, dims, 3, coefs=coefs)
    eb = rel_l2(gb, wb)
    say(f"  forward rel-L2 {e:.3e}, adjoint rel-L2 {eb:.3e} (blob fit fp32 {blob['rel_fp32']:.2e}, "
        f"bf16 {blob['rel_bf16']:.2e})")
    assert e <= 1e-3 and eb <= 1e-3
