"""Pins for the oracle's basis (O1) and quadrature rule (O2).

The basis of eq. (3) is the tensor-product centred B-spline (Sec. 2.2 of the
paper uses degree 2; the benchmark workloads use degree 3).  The values below
are textbook facts of B-splines, checked against two formulas that share no
code (piecewise polynomial vs truncated powers) and against the defining
convolution beta^n = beta^0 * beta^(n-1).
"""
import numpy as np
import pytest
from scipy import integrate

import oracle


@pytest.mark.parametrize("n,x,val", [
    (3, 0.0, 2.0 / 3.0), (3, 1.0, 1.0 / 6.0), (3, -1.0, 1.0 / 6.0), (3, 2.0, 0.0), (3, -2.5, 0.0),
    (3, 0.5, 23.0 / 48.0), (3, 1.5, 1.0 / 48.0),
    (2, 0.0, 0.75), (2, 0.5, 0.5), (2, -0.5, 0.5), (2, 1.0, 0.125), (2, 1.5, 0.0),
    (1, 0.0, 1.0), (1, 0.5, 0.5), (1, -0.25, 0.75), (1, 1.0, 0.0),
    (0, 0.0, 1.0), (0, 0.49, 1.0), (0, -0.49, 1.0), (0, 0.51, 0.0),
])
def test_known_values(n, x, val):
    assert oracle.bspline(n, [x])[0] == pytest.approx(val, abs=1e-15)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_piecewise_equals_truncated_powers(n):
    rng = np.random.default_rng(11)
    x = rng.uniform(-3, 3, 2000)
    # stay off the knots, where beta^0 conventions differ
    x = x[np.abs(x * 2 - np.round(x * 2)) > 1e-6]
    a = oracle.bspline(n, x)
    b = oracle.bspline(n, x, truncated_power=True)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_partition_of_unity_and_symmetry(n):
    rng = np.random.default_rng(12)
    x = rng.uniform(-5, 5, 300)
    x = x[np.abs(x * 2 - np.round(x * 2)) > 1e-6]
    ks = np.arange(-10, 11)
    s = oracle.bspline(n, (x[:, None] - ks[None, :]).ravel()).reshape(x.size, ks.size).sum(1)
    np.testing.assert_allclose(s, 1.0, atol=1e-14)
    np.testing.assert_allclose(oracle.bspline(n, x), oracle.bspline(n, -x), atol=0)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_unit_integral(n):
    h = 0.5 * (n + 1)
    knots = list(np.arange(-h, h + 0.5, 1.0))
    f = lambda t: oracle.bspline(n, [t])[0]
    val, err = integrate.quad(f, -h - 1, h + 1, points=knots, epsabs=1e-14, limit=200)
    assert val == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_recursive_convolution(n):
    """beta^n(x) = int_{x-1/2}^{x+1/2} beta^(n-1)(t) dt."""
    rng = np.random.default_rng(13)
    hp = 0.5 * n
    knots = list(np.arange(-hp, hp + 0.5, 1.0))
    f = lambda t: oracle.bspline(n - 1, [t])[0]
    for x in rng.uniform(-2.5, 2.5, 25):
        pts = [k for k in knots if x - 0.5 < k < x + 0.5]
        val, _ = integrate.quad(f, x - 0.5, x + 0.5, points=pts or None, epsabs=1e-14)
        assert oracle.bspline(n, [x])[0] == pytest.approx(val, abs=1e-12)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7])
def test_gauss_legendre_rule(m):
    x, w = oracle.gauss_legendre(m)
    xr, wr = np.polynomial.legendre.leggauss(m)
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-15)
    assert w.sum() == pytest.approx(2.0, abs=1e-15)
    for p in range(2 * m):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert (w * x ** p).sum() == pytest.approx(exact, abs=1e-14)
    # degree 2m is not integrated exactly: the rule has the expected order
    assert abs((w * x ** (2 * m)).sum() - 2.0 / (2 * m + 1)) > 1e-6
