"""GPU parity of the quadrature form (exact footprint in FP32) against the
FP64 oracle, through the C ABI.

Bar (exact method evaluated in FP32): relative L2 error <= 1e-5 against the
oracle for projections and back-projections; single footprints within
2e-6 of the largest footprint value.  Edge cases: every degree, anisotropic
volumes, detectors that are not a multiple of the 16 x 16 tile, lines that
graze the volume or miss it, axis-aligned lines (zero slopes), diagonal
lines through lattice edges (dominant-axis ties), a 1 x 1 x 1 volume, a
cone source inside the volume, determinism and independence of how views
are batched.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_11078_amd import synth
from paper_2511_11078_amd.ops import Context, Projector

from gpu_helpers import rel_l2, say, tilted_parallel, to_gpu, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def ctxs():
    return {n: Context(n, "quad", 0) for n in range(4)}


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_footprint_pairs(ctxs, n):
    say(f"footprint pairs n={n}")
    rng = np.random.default_rng(200 + n)
    h = 0.5 * (n + 1)
    w = rng.standard_normal((20000, 3))
    w[np.arange(2000), rng.integers(0, 3, 2000)] = 0.0  # zero slopes
    w[2000:3000] = np.sign(rng.standard_normal((1000, 3)))  # dominant-axis ties
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    x = rng.uniform(-1.6 * h, 1.6 * h, (20000, 3))
    w32 = w.astype(np.float32)
    x32 = x.astype(np.float32)
    got = to_np(ctxs[n].footprint(to_gpu(w32), to_gpu(x32)))
    want = oracle.footprint(n, w32.astype(np.float64) / np.linalg.norm(w32.astype(np.float64), axis=1,
                                                                       keepdims=True), x32.astype(np.float64))
    assert np.count_nonzero(want) > 2000
    err = np.abs(got - want).max()
    say(f"  max abs err {err:.3e} (max value {want.max():.3f})")
    # degree 0 is discontinuous at the support faces: allow the few pairs
    # whose line runs within FP32 rounding of a face to differ
    if n == 0:
        bad = np.abs(got - want) > 2e-6 * want.max()
        assert bad.mean() < 1e-3
    else:
        assert err <= 2e-6 * want.max()


@pytest.mark.parametrize("n", [2, 3])
def test_project_small_parallel_32_full(ctxs, n):
    say(f"project small_parallel_32 n={n}")
    dims = (32, 32, 32)
    c = synth.ellipsoid_phantom(dims, 6, seed=0)
    geom = synth.parallel_geometry(synth.fibonacci_directions(32), 48, 48)
    got = to_np(ctxs[n].project(to_gpu(c), geom))
    want = oracle.project(c, geom, n)
    e = rel_l2(got, want)
    say(f"  rel-L2 {e:.3e}")
    assert e <= TOL


@pytest.mark.parametrize("n", [0, 1, 2, 3])
@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_project_anisotropic_ragged(ctxs, n, kind):
    say(f"project anisotropic {kind} n={n}")
    dims = (40, 24, 16)
    rng = np.random.default_rng(210 + n)
    c = rng.standard_normal(dims[::-1]).astype(np.float32)
    if kind == "parallel":
        geom = tilted_parallel(6, 37, 53, seed=211, pitch=0.9)
    else:
        geom = synth.cone_circular_geometry(6, 29, 61, src_radius=80.0, src_det=120.0, pitch=0.8, angle0=0.37)
    got = to_np(ctxs[n].project(to_gpu(c), geom))
    want = oracle.project(c, geom, n)
    e = rel_l2(got, want)
    say(f"  rel-L2 {e:.3e}")
    # degree 0: lines within rounding of a voxel face may switch voxel
    assert e <= (TOL if n > 0 else 1e-4)


@pytest.mark.parametrize("n", [1, 3])
def test_project_edge_lines(ctxs, n):
    """Axis-aligned, diagonal (ties) and grazing lines, and lines that miss."""
    say(f"project edge lines n={n}")
    dims = (9, 8, 7)
    rng = np.random.default_rng(220)
    c = rng.uniform(0.5, 1.5, dims[::-1]).astype(np.float32)
    dirs = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 0], [1, 1, 1], [1, -1, 1], [0.3, 0.3, 0.9]]
    vecs = []
    for w in dirs:
        w = np.asarray(w, dtype=np.float64)
        w /= np.linalg.norm(w)
        u, v = synth.detector_frame(w)
        vecs.append(np.concatenate([w, [0.0, 0.0, 0.0], 1.0 * u, 1.0 * v]))
    geom = synth.Geometry("parallel", len(dirs), 25, 25, np.asarray(vecs, dtype=np.float32))
    got = to_np(ctxs[n].project(to_gpu(c), geom))
    want = oracle.project(c, geom, n)
    e = rel_l2(got, want)
    say(f"  rel-L2 {e:.3e}")
    assert e <= TOL
    # lines far outside give exactly zero; so do lines that miss the support
    assert np.all(got[want == 0.0] == 0.0)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-5 * scale


def test_project_single_coefficient(ctxs):
    say("project 1x1x1")
    c = np.array([[[2.5]]], dtype=np.float32)
    geom = tilted_parallel(5, 9, 9, seed=230, pitch=0.7)
    for n in (1, 2, 3):
        got = to_np(ctxs[n].project(to_gpu(c), geom))
        want = oracle.project(c, geom, n)
        assert rel_l2(got, want) <= TOL


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("case", ["1x1x1_3x3", "2x1x3_1x1", "1x5x1_1x7"])
def test_minimal_sizes_both_directions(ctxs, n, case):
    """Smallest volumes and detectors: bricks holding a single cell row or
    coefficient, a one-pixel detector, and a single view."""
    say(f"minimal sizes {case} n={n}")
    vol, det = case.split("_")
    dims = tuple(int(t) for t in vol.split("x"))
    R, C = (int(t) for t in det.split("x"))
    rng = np.random.default_rng(270 + n)
    geom = tilted_parallel(1 if case.startswith("2x1x3") else 4, R, C, seed=271, pitch=0.6)
    c = rng.standard_normal(dims[::-1]).astype(np.float32)
    got = to_np(ctxs[n].project(to_gpu(c), geom))
    want = oracle.project(c, geom, n)
    y = rng.standard_normal(want.shape).astype(np.float32)
    gb = to_np(ctxs[n].backproject(to_gpu(y), geom, dims))
    wb = oracle.backproject_subset(y, geom, dims, n)
    e, eb = rel_l2(got, want), rel_l2(gb, wb)
    say(f"  forward rel-L2 {e:.3e}, adjoint rel-L2 {eb:.3e}")
    assert (np.abs(want).max() == 0 or e <= TOL) and (np.abs(wb).max() == 0 or eb <= TOL)
    if np.abs(want).max() == 0:
        assert np.abs(got).max() == 0 and np.abs(gb).max() == 0


@pytest.mark.parametrize("n", [0, 1, 2, 3])
@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_backproject_all_coefficients(ctxs, n, kind):
    say(f"backproject {kind} n={n}")
    dims = (21, 18, 13)
    rng = np.random.default_rng(240 + n)
    if kind == "parallel":
        geom = tilted_parallel(5, 31, 27, seed=241)
    else:
        geom = synth.cone_circular_geometry(5, 23, 35, src_radius=60.0, src_det=90.0, pitch=1.1, angle0=0.2)
    y = rng.standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32)
    got = to_np(ctxs[n].backproject(to_gpu(y), geom, dims))
    want = oracle.backproject_subset(y, geom, dims, n)
    e = rel_l2(got, want)
    say(f"  rel-L2 {e:.3e}")
    assert e <= (TOL if n > 0 else 1e-4)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_forward_copy_choice_by_view_angle(ctxs, n):
    """The forward walks each view in the x- or the y-fastest copy of the
    coefficients, chosen from the angle between the view's central ray and
    its dominant horizontal axis (thresholds 15 and 35 degrees): views on
    both sides of every threshold, in several quadrants, each against the
    oracle; and the allocation-free forward, which runs the same two
    launches, equal bit for bit."""
    say(f"forward copy choice n={n}")
    dims = (13, 11, 9)
    angles = [2, 14, 16, 34, 36, 54, 56, 74, 76, 88, 106, 196]
    one = [synth.cone_circular_geometry(1, 20, 22, src_radius=40.0, src_det=60.0, angle0=np.deg2rad(a))
           for a in angles]
    geom = synth.Geometry("cone", len(angles), 20, 22, np.concatenate([g.vecs for g in one]))

    def walks_yfast(e):  # the kernel's rule, restated to check that both copies are used
        ax, ay, az = np.abs(e[3:6].astype(np.float64) - e[0:3])
        hi, lo = max(ax, ay), min(ax, ay)
        if not az < hi:
            return False
        t = lo / hi
        return t < np.tan(np.deg2rad(15)) if ax >= ay else np.tan(np.deg2rad(15)) <= t < np.tan(np.deg2rad(35))

    side = [walks_yfast(e) for e in geom.vecs]
    assert any(side) and not all(side)
    c = np.random.default_rng(260 + n).uniform(0.0, 1.0, dims[::-1]).astype(np.float32)
    got = to_np(ctxs[n].project(to_gpu(c), geom))
    want = oracle.project(c, geom, n).reshape(got.shape)
    errs = [rel_l2(got[k], want[k]) for k in range(len(angles))]
    say("  per view rel-L2 " + " ".join(f"{a}:{e:.1e}" for a, e in zip(angles, errs)))
    assert max(errs) <= TOL
    from paper_2511_11078_amd.ops import project_noalloc
    assert np.array_equal(to_np(project_noalloc(to_gpu(c), geom, degree=n)), got)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_backproject_z_chunks_match_one_pass(n):
    """A scratch limit below the knot-cell table splits the adjoint into
    z-chunks of 4 (n+1) cell layers (the floor) that overlap by n layers:
    the result matches the one-pass adjoint to FP32 rounding (the cell
    bricks align to each chunk's first layer, so line set-ups round
    differently; a lost or doubled layer would differ by O(1)), and the
    oracle on every coefficient.  A ragged last chunk (the layer count is not
    a multiple of the chunk step) and a default limit restored afterwards."""
    say(f"backproject z-chunks n={n}")
    dims = (23, 19, 61)
    geom = synth.cone_circular_geometry(6, 29, 33, src_radius=80.0, src_det=120.0, pitch=1.7, angle0=0.4)
    y = np.random.default_rng(250 + n).standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32)
    one = Context(n, "quad", 0)
    chunked = Context(n, "quad", 0)
    chunked.set_scratch_limit(1)
    b1 = to_np(one.backproject(to_gpu(y), geom, dims))
    bc = to_np(chunked.backproject(to_gpu(y), geom, dims))
    e_pass = rel_l2(bc, b1)
    e_oracle = rel_l2(bc, oracle.backproject_subset(y, geom, dims, n))
    chunked.set_scratch_limit(0)
    bd = to_np(chunked.backproject(to_gpu(y), geom, dims))
    say(f"  chunked vs one pass {e_pass:.2e}, vs oracle {e_oracle:.2e}, default again {rel_l2(bd, b1):.1e}")
    assert e_pass <= 2e-6
    assert e_oracle <= (TOL if n > 0 else 1e-4)
    assert np.array_equal(bd, b1)
    one.close()
    chunked.close()


@pytest.mark.parametrize("case", ["cone_fine_pitch", "parallel_wide_rows"])
def test_backproject_large_shadows(ctxs, case):
    """Detector pixels much smaller than a knot cell: a brick's shadow holds
    more lines than the LDS table (rows split into segments; in the second
    case a single row is wider than the table, so columns split too) and a
    cell is hit by far more lines per view than a thread queues at once."""
    say(f"backproject large shadows: {case}")
    rng = np.random.default_rng(245)
    if case == "cone_fine_pitch":
        dims = (17, 15, 11)
        geom = synth.cone_circular_geometry(3, 150, 170, src_radius=40.0, src_det=60.0, pitch=0.16, angle0=0.3)
    else:
        # columns along the diagonal of the x1-x2 plane, so that an 8 x 8
        # brick spans all 900 columns (more than the table holds)
        dims = (9, 5, 4)
        vecs = []
        for tilt in (0.1, -0.07):
            w = np.array([tilt, 0.05, 1.0])
            w /= np.linalg.norm(w)
            u = np.array([1.0, 1.0, 0.0])
            u -= (u @ w) * w
            u /= np.linalg.norm(u)
            vecs.append(np.concatenate([w, np.zeros(3), 0.012 * u, 0.012 * np.cross(w, u)]))
        geom = synth.Geometry("parallel", 2, 40, 900, np.asarray(vecs, dtype=np.float32))
    y = rng.standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32)
    coefs = synth.sample_indices(int(np.prod(dims)), 120, seed=247)
    got = to_np(ctxs[3].backproject(to_gpu(y), geom, dims)).ravel()[coefs]
    want = oracle.backproject_subset(y, geom, dims, 3, coefs=coefs)
    e = rel_l2(got, want)
    say(f"  rel-L2 {e:.3e} over {coefs.size} coefficients")
    assert np.abs(want).max() > 0 and e <= TOL


@pytest.mark.parametrize("n", [2, 3])
def test_source_inside_volume(ctxs, n):
    """Cone source inside the volume (the whole line is integrated, so cells
    behind the source are hit too).  Bricks with a corner on or behind the
    source plane take every pixel of the detector as candidates: several
    table segments per view, a switch of table halves within a view and a
    per-thread queue that overflows and wraps many times."""
    say(f"source inside the volume n={n}")
    rng = np.random.default_rng(260 + n)
    dims = (13, 11, 9)
    geom = synth.cone_circular_geometry(3, 24, 26, src_radius=3.0, src_det=12.0, angle0=0.4)
    c = rng.standard_normal(dims[::-1]).astype(np.float32)
    got = to_np(ctxs[n].project(to_gpu(c), geom))
    want = oracle.project(c, geom, n)
    e = rel_l2(got, want)
    y = rng.standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32)
    gb = to_np(ctxs[n].backproject(to_gpu(y), geom, dims))
    wb = oracle.backproject_subset(y, geom, dims, n)
    eb = rel_l2(gb, wb)
    say(f"  forward rel-L2 {e:.3e}, adjoint rel-L2 {eb:.3e}")
    assert e <= TOL and eb <= TOL


@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_dot_product_test(ctxs, kind):
    say(f"dot test {kind}")
    dims = (33, 30, 28)
    rng = np.random.default_rng(250)
    if kind == "parallel":
        geom = tilted_parallel(7, 45, 47, seed=251)
    else:
        geom = synth.cone_circular_geometry(7, 41, 49, src_radius=80.0, src_det=120.0, angle0=0.1)
    x = to_gpu(rng.standard_normal(dims[::-1]).astype(np.float32))
    y = to_gpu(rng.standard_normal((geom.n_views, geom.det_rows, geom.det_cols)).astype(np.float32))
    ctx = ctxs[3]
    Ax = ctx.project(x, geom)
    Aty = ctx.backproject(y, geom, dims)
    lhs = float((Ax.double() * y.double()).sum())
    rhs = float((x.double() * Aty.double()).sum())
    rel = abs(lhs - rhs) / (float(Ax.double().norm()) * float(y.double().norm()))
    say(f"  dot-test relative mismatch {rel:.3e}")
    assert rel <= 1e-5


def test_deterministic_and_batch_invariant(ctxs):
    say("determinism / view batching")
    dims = (30, 26, 22)
    rng = np.random.default_rng(260)
    c = to_gpu(rng.standard_normal(dims[::-1]).astype(np.float32))
    geom = synth.cone_circular_geometry(12, 33, 39, src_radius=70.0, src_det=105.0, angle0=0.5)
    ctx = ctxs[3]
    y1 = ctx.project(c, geom).clone()
    y2 = ctx.project(c, geom).clone()
    assert torch.equal(y1, y2)
    parts = [ctx.project(c, geom.subset_views(v0, min(v0 + 5, 12))).clone() for v0 in range(0, 12, 5)]
    assert torch.equal(torch.cat(parts, 0), y1)
    b1 = ctx.backproject(y1, geom, dims).clone()
    b2 = ctx.backproject(y1, geom, dims).clone()
    assert torch.equal(b1, b2)


def test_projector_autograd_backward_is_adjoint(ctxs):
    say("autograd wiring")
    from paper_2511_11078_amd.ops import Project
    dims = (20, 17, 15)
    geom = tilted_parallel(4, 25, 23, seed=270)
    P = Projector(dims, geom, context=ctxs[3])
    rng = np.random.default_rng(271)
    c = to_gpu(rng.standard_normal(dims[::-1]).astype(np.float32)).requires_grad_(True)
    g = to_gpu(rng.standard_normal(P.sino_shape).astype(np.float32))
    y = Project.apply(c, P)
    y.backward(g)
    assert torch.equal(c.grad, P.adjoint(g))
