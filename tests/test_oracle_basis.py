"""Pins for the oracle's 1-D bases against independent library routines and identities."""
import numpy as np
import pytest
from scipy.interpolate import BPoly, BSpline

from oracle.basis import bernstein, bspline_basis, gauss01, support_elements


KNOTS = [
    (2, np.array([0, 0, 0, .5, 1, 1, 1.])),
    (3, np.array([0, 0, 0, 0, .2, .45, .7, 1, 1, 1, 1.])),
    (2, np.array([0, 0, 0, .3, .3, .8, 1, 1, 1.])),      # repeated interior knot
    (1, np.array([0, 0, .25, .5, 1, 1.])),
    (4, np.array([0] * 5 + [.5] + [1] * 5, dtype=float)),
    (0, np.array([0, .4, 1.])),
]


@pytest.mark.parametrize("p,t", KNOTS)
def test_bspline_matches_scipy(p, t):
    x = np.linspace(0, 1, 57)[:-1] + 0.003
    N, dN = bspline_basis(t, p, x, deriv=True)
    n = len(t) - p - 1
    for i in range(n):
        c = np.zeros(n)
        c[i] = 1.0
        s = BSpline(t, c, p, extrapolate=False)
        np.testing.assert_allclose(N[:, i], s(x), atol=1e-14)
        if p > 0:
            np.testing.assert_allclose(dN[:, i], s.derivative()(x), atol=1e-12)


@pytest.mark.parametrize("p,t", KNOTS)
def test_partition_of_unity_and_right_end(p, t):
    x = np.concatenate([np.linspace(0, 1, 31), [1.0]])
    N, dN = bspline_basis(t, p, x, deriv=True)
    np.testing.assert_allclose(N.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(dN.sum(axis=1), 0.0, atol=1e-12)
    assert N[-1, -1] == pytest.approx(1.0)


def test_support_elements():
    p, t = KNOTS[1]
    sup = support_elements(t, p)
    x = np.linspace(0, 1, 400)[1:-1]
    N = bspline_basis(t, p, x)
    spans = [(t[i], t[i + 1]) for i in range(len(t) - 1) if t[i] < t[i + 1]]
    for i, s in enumerate(sup):
        for e, (lo, hi) in enumerate(spans):
            inside = (x > lo) & (x < hi)
            assert (np.abs(N[inside, i]).max() > 0) == (e in s)


@pytest.mark.parametrize("q", [0, 1, 2, 3, 5])
def test_bernstein_matches_scipy_bpoly(q):
    x = np.linspace(0, 1, 41)
    B, dB = bernstein(q, x, deriv=True)
    for c in range(q + 1):
        coef = np.zeros((q + 1, 1))
        coef[c, 0] = 1.0
        bp = BPoly(coef, [0.0, 1.0])
        np.testing.assert_allclose(B[:, c], bp(x), atol=1e-14)
        if q > 0:
            np.testing.assert_allclose(dB[:, c], bp.derivative()(x), atol=1e-12)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_gauss_exactness(n):
    x, w = gauss01(n)
    for d in range(2 * n):
        assert np.dot(w, x ** d) == pytest.approx(1.0 / (d + 1), abs=1e-14)
