"""Pins for the lookup table (eq. (51)-(57)) and the pair set I_coo."""
import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import BPoly, BSpline

import workloads as W
from oracle import tables


def _pairs_count_closed_form(tile):
    """|I_coo| = (X + n_T)/2 with X the number of ordered 3-D pairs, the product of 1-D counts
    of |i - j| <= p (uniform clamped knots, no repeated interior knots)."""
    X = 1
    for k in range(3):
        n = tile.n_ctrl[k]
        p = tile.degree[k]
        X *= sum(1 for i in range(n) for j in range(n) if abs(i - j) <= p)
    nT = int(np.prod(tile.n_ctrl))
    return (X + nT) // 2


@pytest.mark.parametrize("name,expect", [("cfg1", 1404), ("cfg2", 25498), ("cfg3", 3492)])
def test_pair_counts(name, expect):
    w = W.make(name) if name != "cfg3" else W.make("cfg3", n_el=2)
    pairs = tables.pair_set(w.tile)
    assert len(pairs) == expect == _pairs_count_closed_form(w.tile)
    assert np.all(pairs[:, 0] <= pairs[:, 1])
    key = pairs[:, 0] * 10 ** 6 + pairs[:, 1]
    assert np.all(np.diff(key) > 0)


@pytest.fixture(scope="module")
def cfg1_tables():
    w = W.make("cfg1")
    pairs = tables.pair_set(w.tile)
    return w, pairs, {q: tables.stiffness_table(w.tile, q, 3, pairs) for q in range(4)}


def _full(table, pairs, nT, npi):
    """K(A, B, C, i, j) for all ordered (A, B) using K(B, A, C, i, j) = K(A, B, C, j, i)."""
    K = np.zeros((nT, nT, npi, 3, 3))
    T = table.reshape(len(pairs), npi, 3, 3)
    K[pairs[:, 0], pairs[:, 1]] = T
    K[pairs[:, 1], pairs[:, 0]] = T.transpose(0, 1, 3, 2)
    return K


def test_row_sums_vanish(cfg1_tables):
    """sum_B d_j(R_B o T^-1) = 0, so sum_B K(A,B,C,i,j) = 0 for every A, C, i, j."""
    w, pairs, T = cfg1_tables
    nT = 64
    for q in (0, 2):
        K = _full(T[q], pairs, nT, (q + 1) ** 3)
        s = np.abs(K.sum(axis=1)).max()
        assert s < 1e-13 * np.abs(K).max()


def test_bernstein_sum_gives_degree_zero_table(cfg1_tables):
    w, pairs, T = cfg1_tables
    for q in (1, 2, 3):
        Tq = T[q].reshape(len(pairs), (q + 1) ** 3, 9).sum(axis=1)
        np.testing.assert_allclose(Tq, T[0], atol=1e-14 * np.abs(T[0]).max())


def _elevation(q):
    E = np.zeros((q + 1, q + 2))
    for c in range(q + 1):
        E[c, c] = (q + 1 - c) / (q + 1)
        E[c, c + 1] = (c + 1) / (q + 1)
    return np.einsum("ad,be,cf->cbafed", E, E, E).reshape((q + 1) ** 3, (q + 2) ** 3)


def test_degree_elevation(cfg1_tables):
    """B^q_c = sum_c' E[c,c'] B^{q+1}_c', so K_q = E3 K_{q+1} column-block-wise."""
    w, pairs, T = cfg1_tables
    for q in (0, 1, 2):
        E3 = _elevation(q)
        a = T[q].reshape(len(pairs), (q + 1) ** 3, 9)
        b = np.einsum("CD,pDk->pCk", E3, T[q + 1].reshape(len(pairs), (q + 2) ** 3, 9))
        np.testing.assert_allclose(a, b, atol=1e-14 * np.abs(a).max())


def test_diagonal_pair_symmetry(cfg1_tables):
    w, pairs, T = cfg1_tables
    d = pairs[:, 0] == pairs[:, 1]
    blk = T[2].reshape(len(pairs), 27, 3, 3)[d]
    np.testing.assert_allclose(blk, blk.transpose(0, 1, 3, 2), atol=1e-15 * np.abs(blk).max())


def _oned_integral(t, p, a, b, c, q, da, db):
    ca = np.zeros(len(t) - p - 1); ca[a] = 1
    cb = np.zeros(len(t) - p - 1); cb[b] = 1
    ra = BSpline(t, ca, p)
    rb = BSpline(t, cb, p)
    if da:
        ra = ra.derivative()
    if db:
        rb = rb.derivative()
    coef = np.zeros((q + 1, 1)); coef[c, 0] = 1
    bern = BPoly(coef, [0.0, 1.0])
    brk = np.unique(t)
    tot = 0.0
    for lo, hi in zip(brk[:-1], brk[1:]):
        tot += integrate.quad(lambda x: ra(x) * rb(x) * bern(x), lo, hi, epsabs=1e-16, epsrel=1e-13, limit=200)[0]
    return tot


def test_identity_tile_separable_integrals():
    """For the identity tile the integrand of eq. (52) is a product of 1-D factors:
    K(A,B,C,i,j) = prod_k int r_{a_k}^(d_ik) r_{b_k}^(d_jk) B_{c_k}, computed with scipy's BSpline/BPoly/quad.
    The 1-D integrands have degree <= 2 p + q = 6, so 4 Gauss points per element are exact."""
    tile = W.identity_spline((2, 2, 2), (2, 2, 2))
    q = 2
    pairs = tables.pair_set(tile)
    T = tables.stiffness_table(tile, q, 4, pairs).reshape(len(pairs), 27, 3, 3)
    t = tile.knots[0]
    rng = np.random.default_rng(5)
    for p in rng.choice(len(pairs), size=25, replace=False):
        A, B = pairs[p]
        ai = (A % 4, (A // 4) % 4, A // 16)
        bi = (B % 4, (B // 4) % 4, B // 16)
        for C in rng.choice(27, size=3, replace=False):
            ci = (C % 3, (C // 3) % 3, C // 9)
            for i in range(3):
                for j in range(3):
                    val = 1.0
                    for k in range(3):
                        val *= _oned_integral(t, 2, ai[k], bi[k], ci[k], q, i == k, j == k)
                    assert T[p, C, i, j] == pytest.approx(val, abs=1e-13)
