"""Pins for the oracle's operators: O3 (direct integral), O5 (basis sum),
O6 (voxel-driven transpose), O7 (dense matrix), O8 (CGLS), O9 (counts).

Each test checks the oracle against something other than itself:
closed forms (axis-aligned views reduce to a 2-D spline evaluation of column
sums; partition of unity turns an all-ones volume into the interior chord
length), brute-force adaptive quadrature of f along a line with an
independent evaluation of f, two exact formulations of the same transform
(direct integral vs sum of footprints, eq. (4)), equivariances, linearity,
the dot-product test for the transpose and textbook CG for CGLS.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2511_11078_amd import synth


def _beta3(x):
    a = np.abs(x)
    return np.where(a < 1, 2 / 3 - a * a + a ** 3 / 2, np.where(a < 2, (2 - a) ** 3 / 6, 0.0))


def _beta2(x):
    a = np.abs(x)
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


BETA = {2: _beta2, 3: _beta3}


def _axis_geometry(d, R, C, d0):
    """One parallel view along +e_d; columns step along the next axis, rows
    along the one after."""
    i, j = (d + 1) % 3, (d + 2) % 3
    vec = np.zeros(12)
    vec[d] = 1.0
    vec[3:6] = d0
    vec[6 + i] = 1.0
    vec[9 + j] = 1.0
    return synth.Geometry("parallel", 1, R, C, vec[None].astype(np.float32)), i, j


@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_axis_aligned_view_is_2d_spline_of_column_sums(n, d):
    dims = (7, 5, 4)  # N1, N2, N3 -- anisotropic to catch axis mix-ups
    rng = np.random.default_rng(100 + d)
    c = rng.standard_normal(dims[::-1]).astype(np.float32)  # [N3, N2, N1]
    R, C = 9, 11
    d0 = np.array([0.31, -0.17, 0.23]).astype(np.float32).astype(np.float64)
    geom, i, j = _axis_geometry(d, R, C, d0)
    y = oracle.project(c, geom, n)[0]
    # independent closed form: S[k_j, k_i] = sum over k_d of c, then a 2-D spline
    carr = c.astype(np.float64).transpose(2, 1, 0)  # [k1, k2, k3]
    S = carr.sum(axis=d)
    axes = [a for a in range(3) if a != d]
    xk = [np.arange(dims[a]) - 0.5 * (dims[a] - 1) for a in range(3)]
    want = np.zeros((R, C))
    for jj in range(R):
        for ii in range(C):
            p = d0.copy()
            p[i] += ii - 0.5 * (C - 1)
            p[j] += jj - 0.5 * (R - 1)
            b = {a: BETA[n](p[a] - xk[a]) for a in axes}
            want[jj, ii] = b[axes[0]] @ S @ b[axes[1]]
    np.testing.assert_allclose(y, want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("n", [1, 2, 3])
def test_all_ones_gives_interior_chord_length(n):
    dims = (40, 40, 8)
    c = np.ones(dims[::-1], dtype=np.float32)
    dirs = np.array([[0.0, 0.0, 1.0], [0.05, 0.03, 1.0], [-0.04, 0.02, 1.0]])
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    vecs = np.zeros((3, 12))
    vecs[:, 0:3] = dirs
    vecs[:, 3:6] = [0.37, -0.21, 0.0]
    vecs[:, 6] = 1.0
    vecs[:, 10] = 1.0
    geom = synth.Geometry("parallel", 3, 3, 3, vecs.astype(np.float32))
    y = oracle.project(c, geom, n)
    geom_w = oracle.make_rays(geom)[1].reshape(3, 9, 3)[:, 0, 2]
    want = 8.0 / np.abs(geom_w)
    np.testing.assert_allclose(y.reshape(3, 9), want[:, None] * np.ones((1, 9)), rtol=1e-12)


def _f_point(c, n, x):
    """Independent evaluation of f(x) = sum_k c_k phi(x - x_k)."""
    N3, N2, N1 = c.shape
    xk = [np.arange(N) - 0.5 * (N - 1) for N in (N1, N2, N3)]
    b = [BETA[n](x[a] - xk[a]) for a in range(3)]
    return float(np.einsum("kji,i,j,k->", c.astype(np.float64), b[0], b[1], b[2]))


# quad may report that round-off keeps it from its 1e-12 target on the
# piecewise-polynomial integrand; the comparison below asks for 1e-9 only
@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("n", [2, 3])
def test_direct_integral_vs_brute_force_quadrature(n):
    rng = np.random.default_rng(110 + n)
    c = rng.standard_normal((3, 4, 5)).astype(np.float32)
    geom = synth.parallel_geometry(synth.uniform_directions(4, seed=111), 3, 3)
    y = oracle.project(c, geom, n).ravel()
    a, w = oracle.make_rays(geom)
    for r in range(0, y.size, 2):
        f = lambda t: _f_point(c, n, a[r] + t * w[r])
        val, _ = integrate.quad(f, -12, 12, limit=4000, epsabs=1e-13, epsrel=1e-12)
        assert y[r] == pytest.approx(val, abs=1e-9)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_direct_integral_equals_basis_sum(n, kind):
    rng = np.random.default_rng(120 + n)
    dims = (9, 7, 6)
    c = rng.standard_normal(dims[::-1]).astype(np.float32)
    if kind == "parallel":
        geom = synth.parallel_geometry(synth.uniform_directions(5, seed=121), 10, 12, pitch=0.9)
    else:
        geom = synth.cone_circular_geometry(5, 10, 12, src_radius=25.0, src_det=37.5, pitch=1.1,
                                            angle0=0.3)
    y3 = oracle.project(c, geom, n)
    y5 = oracle.project_basis_sum(c, geom, n)
    scale = np.abs(y3).max()
    np.testing.assert_allclose(y5, y3, rtol=0, atol=1e-12 * scale)
    assert np.count_nonzero(y3) > y3.size // 4


@pytest.mark.parametrize("n", [2, 3])
def test_shift_equivariance(n):
    rng = np.random.default_rng(130)
    dims = (8, 7, 6)
    c = rng.standard_normal(dims[::-1]).astype(np.float32)
    c[-1, :, :] = 0
    c[:, -1, :] = 0
    c[:, :, -1] = 0
    geom = synth.parallel_geometry(synth.uniform_directions(3, seed=131), 6, 6)
    y = oracle.project(c, geom, n)
    for axis in range(3):  # world axis
        cs = np.roll(c, 1, axis=2 - axis)
        g2 = synth.Geometry("parallel", geom.n_views, 6, 6, geom.vecs.copy())
        g2.vecs[:, 3 + axis] += 1.0
        ys = oracle.project(cs, g2, n)
        np.testing.assert_allclose(ys, y, atol=1e-12 * np.abs(y).max())


@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_axis_permutation_equivariance(kind):
    rng = np.random.default_rng(140)
    dims = (9, 6, 5)
    c = rng.standard_normal(dims[::-1]).astype(np.float32)
    if kind == "parallel":
        geom = synth.parallel_geometry(synth.uniform_directions(3, seed=141), 7, 8)
    else:
        geom = synth.cone_circular_geometry(3, 7, 8, 20.0, 30.0, angle0=0.2)
    y = oracle.project(c, geom, 3)
    # swap world axes 1 and 3: array [N3, N2, N1] -> [N1, N2, N3]
    cT = np.ascontiguousarray(c.transpose(2, 1, 0))
    vT = geom.vecs.reshape(-1, 4, 3)[:, :, ::-1].reshape(-1, 12).copy()
    gT = synth.Geometry(kind, geom.n_views, 7, 8, vT)
    yT = oracle.project(cT, gT, 3)
    np.testing.assert_allclose(yT, y, atol=1e-12 * np.abs(y).max())


def test_linearity():
    rng = np.random.default_rng(150)
    dims = (6, 6, 6)
    c1 = rng.standard_normal(dims).astype(np.float32)
    c2 = rng.standard_normal(dims).astype(np.float32)
    geom = synth.parallel_geometry(synth.fibonacci_directions(4), 5, 5)
    a = np.float32(0.75)
    b = np.float32(-1.5)
    lhs = oracle.project((a * c1 + b * c2).astype(np.float32), geom, 3)
    rhs = float(a) * oracle.project(c1, geom, 3) + float(b) * oracle.project(c2, geom, 3)
    # c' = a c1 + b c2 is rounded to FP32 before projection
    assert np.abs(lhs - rhs).max() <= 1e-6 * np.abs(rhs).max()


def test_cone_rays_match_hand_built_lines():
    geom = synth.cone_circular_geometry(4, 5, 6, src_radius=30.0, src_det=45.0, pitch=1.3, angle0=0.4)
    a, w = oracle.make_rays(geom)
    vecs = geom.vecs.astype(np.float64)
    r = 0
    for v in range(4):
        s, d0, du, dv = vecs[v, 0:3], vecs[v, 3:6], vecs[v, 6:9], vecs[v, 9:12]
        for j in range(5):
            for i in range(6):
                p = d0 + (i - 2.5) * du + (j - 2.0) * dv
                d = (p - s) / np.linalg.norm(p - s)
                np.testing.assert_allclose(w[r], d, atol=1e-15)
                # the anchor lies on the same line
                off = a[r] - s
                assert np.linalg.norm(off - (off @ d) * d) < 1e-12
                r += 1
    # a cone view equals the parallel views built from its lines
    rng = np.random.default_rng(160)
    c = rng.standard_normal((6, 7, 8)).astype(np.float32)
    y = oracle.project(c, geom, 3).ravel()
    pv = np.zeros((a.shape[0], 12))
    pv[:, 0:3] = w
    pv[:, 3:6] = a
    pv[:, 6] = 1.0
    pv[:, 10] = 1.0
    gp = synth.Geometry("parallel", a.shape[0], 1, 1, pv.astype(np.float32))
    yp = oracle.project(c, gp, 3).ravel()
    # the float32 rounding of the hand-built vectors moves the lines by ~1e-7
    np.testing.assert_allclose(yp, y, atol=1e-5 * np.abs(y).max())


@pytest.mark.parametrize("n", [0, 2, 3])
@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_adjoint_dot_product_and_dense_transpose(n, kind):
    rng = np.random.default_rng(170 + n)
    dims = (8, 7, 6)
    if kind == "parallel":
        geom = synth.parallel_geometry(synth.uniform_directions(4, seed=171), 9, 10, pitch=0.8)
    else:
        geom = synth.cone_circular_geometry(4, 9, 10, 20.0, 30.0, pitch=1.2, angle0=0.1)
    x = rng.standard_normal(dims[::-1]).astype(np.float32)
    y = rng.standard_normal((geom.n_views, 9, 10)).astype(np.float32)
    Ax = oracle.project(x, geom, n)
    Aty = oracle.backproject_subset(y, geom, dims, n)
    lhs = float((Ax * y.astype(np.float64)).sum())
    rhs = float((x.astype(np.float64) * Aty).sum())
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)
    A = oracle.dense_matrix(dims, geom, n)
    np.testing.assert_allclose(A @ x.astype(np.float64).ravel(), Ax.ravel(), atol=1e-12 * np.abs(Ax).max())
    np.testing.assert_allclose(A.T @ y.astype(np.float64).ravel(), Aty.ravel(), atol=1e-12 * np.abs(Aty).max())
    # subset evaluation equals the full one
    sub = synth.sample_indices(x.size, 37, seed=172)
    np.testing.assert_allclose(oracle.backproject_subset(y, geom, dims, n, coefs=sub), Aty.ravel()[sub], atol=0)
    # pair counts equal the non-zero pattern of the matrix rows (degree >= 1)
    if n > 0:
        pairs, segs = oracle.counts(dims, geom, n)
        np.testing.assert_array_equal(pairs, np.count_nonzero(A, axis=1))
        assert np.all(segs >= pairs) and np.all(segs <= (3 * n + 1) * pairs)


def test_cgls_matches_textbook_cg_and_lstsq():
    rng = np.random.default_rng(180)
    dims = (5, 5, 4)
    geom = synth.parallel_geometry(synth.fibonacci_directions(12), 8, 8)
    A = oracle.dense_matrix(dims, geom, 3)
    x_true = rng.standard_normal(A.shape[1])
    y = A @ x_true + 0.01 * rng.standard_normal(A.shape[0])
    # iterate-by-iterate agreement holds while the Krylov basis is well
    # conditioned; beyond ~12 steps both recurrences drift by round-off
    iters = 10
    x, hist = oracle.cgls(lambda v: A @ v, lambda r: A.T @ r, y, iters)
    # CG on the normal equations A^T A x = A^T y, written out independently
    M = A.T @ A
    b = A.T @ y
    xc = np.zeros_like(b)
    rc = b.copy()
    pc = rc.copy()
    for _ in range(iters):
        Mp = M @ pc
        al = (rc @ rc) / (pc @ Mp)
        xc = xc + al * pc
        rn = rc - al * Mp
        pc = rn + (rn @ rn) / (rc @ rc) * pc
        rc = rn
    np.testing.assert_allclose(x, xc, atol=1e-9 * np.abs(xc).max())
    x, hist = oracle.cgls(lambda v: A @ v, lambda r: A.T @ r, y, 40)
    res = [h[0] for h in hist]
    iters = 40
    assert all(res[k + 1] <= res[k] * (1 + 1e-12) for k in range(iters))
    x_long, _ = oracle.cgls(lambda v: A @ v, lambda r: A.T @ r, y, 400)
    x_ls = np.linalg.lstsq(A, y, rcond=None)[0]
    np.testing.assert_allclose(A @ x_long, A @ x_ls, atol=1e-8 * np.abs(A @ x_ls).max())


@pytest.mark.parametrize("n", [0, 2, 3])
def test_direct_segment_counts(n):
    """An axis-aligned line inside the volume crosses every knot cell of the
    padded box along its axis: N + n + 1 cells (the padded box spans
    N - 1 + 2h = N + n units, bounded by knot planes); an oblique line
    crosses one more cell per knot plane of each other axis."""
    dims = (6, 7, 8)
    vecs = np.zeros((2, 12))
    vecs[0, 0:3] = [0.0, 0.0, 1.0]
    vecs[0, 3:6] = [0.13, -0.21, 0.0]
    vecs[0, 6] = 1.0
    vecs[0, 10] = 1.0
    w = np.array([0.1, 0.05, 1.0])
    vecs[1, 0:3] = w / np.linalg.norm(w)
    vecs[1, 3:6] = [0.13, -0.21, 0.0]
    vecs[1, 6] = 1.0
    vecs[1, 10] = 1.0
    geom = synth.Geometry("parallel", 2, 1, 1, vecs.astype(np.float32))
    segs = oracle.direct_counts(dims, geom, n)
    assert segs[0] == dims[2] + n
    a, ww = oracle.make_rays(geom)
    h = 0.5 * (n + 1)
    kap = 0.0 if n % 2 else 0.5
    # planes crossed by the oblique line inside the padded box
    o = -0.5 * (np.array(dims) - 1)
    lo, hi = o - h, o + np.array(dims) - 1 + h
    t = [(lo[i] - a[1][i]) / ww[1][i] for i in range(3)] + [(hi[i] - a[1][i]) / ww[1][i] for i in range(3)]
    t0 = max(min(t[i], t[i + 3]) for i in range(3))
    t1 = min(max(t[i], t[i + 3]) for i in range(3))
    crossings = 0
    for i in range(3):
        z = sorted([a[1][i] + t0 * ww[1][i] - o[i] - kap, a[1][i] + t1 * ww[1][i] - o[i] - kap])
        crossings += int(np.ceil(z[1]) - np.floor(z[0]) - 1)
    assert segs[1] == crossings + 1
