"""One-dimensional bases used by the method (oracle, test infrastructure only).

* B-spline basis N_{i,p} by the Cox-de Boor recursion (Section 2.2.1, eq. (2)),
  written from its definition for *all* basis functions at once.
* Bernstein polynomials of degree q, the projection basis N^H_C (eq. (21)).
* Gauss-Legendre rule on [0, 1] (NumPy's leggauss, mapped).
"""
from __future__ import annotations

from math import comb

import numpy as np


def n_basis(knots: np.ndarray, p: int) -> int:
    return len(knots) - p - 1


def bspline_basis(knots: np.ndarray, p: int, x, deriv: bool = False):
    """Values (and first derivatives) of all B-spline basis functions at points x.

    Degree-0 functions are indicators of the half-open spans [t_i, t_{i+1});
    the right end of the parameter domain is attached to the last non-empty span.
    Higher degrees follow the Cox-de Boor recursion with 0/0 := 0; the derivative
    is p/(t_{i+p}-t_i) N_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) N_{i+1,p-1}.
    Returns N of shape (len(x), n) and, if deriv, dN of the same shape.
    """
    t = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(t) - 1
    N = np.zeros((x.size, m))
    nonempty = [i for i in range(m) if t[i] < t[i + 1]]
    for i in nonempty:
        N[:, i] = ((t[i] <= x) & (x < t[i + 1])).astype(np.float64)
    N[x >= t[-1], nonempty[-1]] = 1.0
    Nprev = N
    for k in range(1, p + 1):
        Nk = np.zeros((x.size, m - k))
        for i in range(m - k):
            d1 = t[i + k] - t[i]
            d2 = t[i + k + 1] - t[i + 1]
            if d1 > 0:
                Nk[:, i] += (x - t[i]) / d1 * N[:, i]
            if d2 > 0:
                Nk[:, i] += (t[i + k + 1] - x) / d2 * N[:, i + 1]
        Nprev, N = N, Nk
    if not deriv:
        return N
    n = m - p
    dN = np.zeros((x.size, n))
    if p > 0:
        for i in range(n):
            d1 = t[i + p] - t[i]
            d2 = t[i + p + 1] - t[i + 1]
            if d1 > 0:
                dN[:, i] += p / d1 * Nprev[:, i]
            if d2 > 0:
                dN[:, i] -= p / d2 * Nprev[:, i + 1]
    return N, dN


def bernstein(q: int, x, deriv: bool = False):
    """Bernstein polynomials B^q_c(x) = C(q,c) x^c (1-x)^(q-c), c = 0..q, shape (len(x), q+1)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    B = np.stack([comb(q, c) * x ** c * (1.0 - x) ** (q - c) for c in range(q + 1)], axis=1)
    if not deriv:
        return B
    if q == 0:
        return B, np.zeros_like(B)
    Bm = np.stack([comb(q - 1, c) * x ** c * (1.0 - x) ** (q - 1 - c) for c in range(q)], axis=1)
    dB = np.zeros_like(B)
    for c in range(q + 1):
        if c > 0:
            dB[:, c] += q * Bm[:, c - 1]
        if c < q:
            dB[:, c] -= q * Bm[:, c]
    return B, dB


def gauss01(n: int):
    """n-point Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def nonempty_spans(knots: np.ndarray):
    """List of (left, right) for the knot spans of positive length."""
    t = np.asarray(knots)
    return [(t[i], t[i + 1]) for i in range(len(t) - 1) if t[i] < t[i + 1]]


def support_elements(knots: np.ndarray, p: int):
    """For every basis function, the set of non-empty span indices on which it is non-zero."""
    t = np.asarray(knots)
    spans = [i for i in range(len(t) - 1) if t[i] < t[i + 1]]
    out = []
    for i in range(n_basis(t, p)):
        out.append({e for e, s in enumerate(spans) if t[i] <= t[s] and t[s + 1] <= t[i + p + 1]})
    return out
