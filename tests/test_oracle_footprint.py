"""Pins for the oracle's single-basis footprint O4: P phi(w, x) = int phi(x + t w) dt.

The footprint is the "contribution" of one basis to one line (eq. (4) of the
paper).  It has no printed values in the paper, so it is pinned to facts the
mathematics fixes:

* an axis-aligned line through beta^n x beta^n x beta^n gives the product of
  the two transverse factors (int beta^n = 1);
* integrating the footprint over the plane perpendicular to w gives
  int phi = 1;
* projection-slice theorem: its 2-D Fourier transform at xi perpendicular to w
  is phi^(xi) = prod_i sinc^(n+1)(xi_i / 2);
* invariance under the 48 signed permutations (phi is invariant under them);
* degree 0: the chord length of the unit cube;
* brute-force adaptive quadrature of the integrand with no breakpoints;
* zero at and beyond the support.
"""
import itertools

import numpy as np
import pytest
from scipy import integrate

import oracle


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def _frame(w):
    a = np.argmin(np.abs(w))
    e = np.zeros(3)
    e[a] = 1.0
    u = _unit(e - w[a] * w)
    return u, np.cross(w, u)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_axis_aligned_is_product_of_transverse_factors(n, d):
    rng = np.random.default_rng(20 + n)
    x = rng.uniform(-2.6, 2.6, (200, 3))
    w = np.zeros(3)
    w[d] = -1.0 if n % 2 else 1.0
    got = oracle.footprint(n, w, x)
    o = [i for i in range(3) if i != d]
    want = oracle.bspline(n, x[:, o[0]]) * oracle.bspline(n, x[:, o[1]])
    np.testing.assert_allclose(got, want, atol=1e-14)


def _plane_quadrature(n, w, func, panel=0.05, order=4):
    """Composite Gauss-Legendre over the square [-R, R]^2 of the plane w^perp."""
    h = 0.5 * (n + 1)
    R = h * np.sqrt(3.0) + 0.05
    npan = int(np.ceil(2 * R / panel))
    edges = np.linspace(-R, R, npan + 1)
    gx, gw = np.polynomial.legendre.leggauss(order)
    mids = 0.5 * (edges[1:] + edges[:-1])
    half = 0.5 * (edges[1:] - edges[:-1])
    pts = (mids[:, None] + half[:, None] * gx[None, :]).ravel()
    wts = (half[:, None] * gw[None, :]).ravel()
    u, v = _frame(w)
    A, B = np.meshgrid(pts, pts, indexing="ij")
    s = A[..., None] * u + B[..., None] * v
    fp = oracle.footprint(n, w, s)
    W = wts[:, None] * wts[None, :]
    return func(fp, A, B, u, v, W)


# degree 0 is discontinuous across the shadow's edge, so its composite rule
# converges only linearly in the panel width: finer panels, looser bound
@pytest.mark.parametrize("n,tol,panel", [(0, 3e-5, 0.01), (1, 1e-8, 0.05), (2, 1e-9, 0.05),
                                         (3, 1e-9, 0.05)])
def test_integral_over_plane_is_one(n, tol, panel):
    rng = np.random.default_rng(30 + n)
    for w in [_unit(rng.standard_normal(3)) for _ in range(3)] + [_unit([1, 1, 1])]:
        tot = _plane_quadrature(n, w, lambda fp, A, B, u, v, W: (fp * W).sum(), panel=panel)
        assert tot == pytest.approx(1.0, abs=tol)


def _sinc(z):
    return np.sinc(z / np.pi)  # numpy's sinc is sin(pi z)/(pi z)


@pytest.mark.parametrize("n,tol,panel", [(0, 3e-5, 0.01), (2, 1e-9, 0.05), (3, 1e-9, 0.05)])
def test_fourier_slice(n, tol, panel):
    rng = np.random.default_rng(40 + n)
    w = _unit(rng.standard_normal(3))
    for kappa, psi in [(0.7, 0.3), (1.5, 1.1), (3.0, 2.0), (4.5, -0.4)]:
        def ft(fp, A, B, u, v, W):
            xi_uv = (kappa * np.cos(psi), kappa * np.sin(psi))
            return (fp * np.cos(xi_uv[0] * A + xi_uv[1] * B) * W).sum()
        got = _plane_quadrature(n, w, ft, panel=panel)
        u, v = _frame(w)
        xi = kappa * (np.cos(psi) * u + np.sin(psi) * v)
        want = np.prod(_sinc(xi / 2.0) ** (n + 1))
        assert got == pytest.approx(want, abs=tol)


@pytest.mark.parametrize("n", [0, 2, 3])
def test_signed_permutation_invariance(n):
    rng = np.random.default_rng(50 + n)
    w = _unit(rng.standard_normal(3))
    x = rng.uniform(-0.6, 0.6, (40, 3)) * (n + 1)
    base = oracle.footprint(n, w, x)
    assert np.count_nonzero(base) > 10
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1.0, -1.0], repeat=3):
            Q = np.zeros((3, 3))
            for i, p in enumerate(perm):
                Q[i, p] = signs[i]
            got = oracle.footprint(n, Q @ w, x @ Q.T)
            np.testing.assert_allclose(got, base, atol=1e-14)
    np.testing.assert_allclose(oracle.footprint(n, -w, x), base, atol=1e-14)


def test_degree0_is_chord_length_of_unit_cube():
    rng = np.random.default_rng(60)
    for _ in range(200):
        w = _unit(rng.standard_normal(3))
        x = rng.uniform(-0.9, 0.9, 3)
        # independent interval intersection of |x_i + t w_i| < 1/2
        lo, hi = -np.inf, np.inf
        for i in range(3):
            a, b = (-0.5 - x[i]) / w[i], (0.5 - x[i]) / w[i]
            lo, hi = max(lo, min(a, b)), min(hi, max(a, b))
        want = max(0.0, hi - lo)
        assert oracle.footprint(0, w, x) == pytest.approx(want, abs=1e-14)
    # fine sampling for one oblique line
    w = _unit([0.3, -0.5, 0.8])
    x = np.array([0.1, 0.05, -0.2])
    t = np.linspace(-3, 3, 2_000_001)
    inside = np.all(np.abs(x[None, :] + t[:, None] * w[None, :]) < 0.5, axis=1)
    assert oracle.footprint(0, w, x) == pytest.approx(inside.sum() * (t[1] - t[0]), abs=1e-5)


# quad reports that round-off keeps it from its 1e-13 target on the kinks of
# the degree-1 integrand; the comparison below asks for 1e-9 only
@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("n", [1, 2, 3])
def test_brute_force_adaptive_quadrature(n):
    rng = np.random.default_rng(70 + n)
    h = 0.5 * (n + 1)
    for _ in range(12):
        w = _unit(rng.standard_normal(3))
        x = rng.uniform(-h, h, 3) * 0.8
        f = lambda t: float(np.prod(oracle.bspline(n, x + t * w)))
        L = 2 * h * np.sqrt(3.0) + 1.0
        val, _ = integrate.quad(f, -L, L, limit=2000, epsabs=1e-14, epsrel=1e-13)
        assert oracle.footprint(n, w, x) == pytest.approx(val, abs=1e-9)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_zero_outside_support(n):
    rng = np.random.default_rng(80 + n)
    h = 0.5 * (n + 1)
    for _ in range(50):
        w = _unit(rng.standard_normal(3))
        u, v = _frame(w)
        ang = rng.uniform(0, 2 * np.pi)
        r = h * np.sqrt(3.0) * rng.uniform(1.0, 2.0)
        x = r * (np.cos(ang) * u + np.sin(ang) * v)
        assert oracle.footprint(n, w, x) == 0.0
    # a line in a face plane of the support, and one just outside it
    w = _unit([0.2, 0.7, 0.1])
    w[0] = 0.0
    w = _unit(w)
    assert oracle.footprint(n, w, [h, 0.0, 0.0]) == 0.0
    assert oracle.footprint(n, w, [h + 1e-9, 0.1, 0.0]) == 0.0
