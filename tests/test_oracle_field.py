"""Pins for the macro field (eq. (37), Appendix A) and the projection (eq. (23)-(24), (42))."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import geometry, projection
from oracle.basis import bernstein
from oracle.macro_field import cartesian_field, lame, macro_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cube_macro_field.txt")


def _read_cube():
    blocks = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        v = [int(s) for s in line.split()]
        blocks[(v[0] - 1, v[1] - 1)] = np.array(v[2:]).reshape(3, 3)
    return blocks


@pytest.mark.parametrize("L,E,nu", [(1.0, 1.0, 0.3), (0.5, 2.0, 0.25), (3.0, 0.7, 0.1)])
def test_cube_closed_form(L, E, nu):
    """Eq. (98)-(99): the fitted coefficients of the cube reproduce the printed structure."""
    lam, mu = lame(E, nu)
    alpha = {0: 0.0, 1: (lam + 2 * mu) * L, 2: mu * L, 3: lam * L}
    for degree in (1, 2):
        macro = W.affine_macro((degree,) * 3, (1, 1, 1), L * np.eye(3), np.zeros(3))
        tile = W.identity_spline((2, 2, 2), (2, 2, 2))
        w = W.Workload("cube", macro, tile, (1, 1, 1), 0, 2, 3, 3, E=E, nu=nu)
        coef = projection.tile_coefficients(w, 0).reshape(27, 3, 3, 3, 3)  # [C, i, j, a, b]
        for (i, j), sym in _read_cube().items():
            expect = np.vectorize(alpha.get)(sym)
            for C in range(27):
                np.testing.assert_allclose(coef[C, i, j], expect, atol=1e-14 * alpha[1])
                np.testing.assert_allclose(coef[C, j, i], expect.T, atol=1e-14 * alpha[1])


def _random_J(rng, n):
    return rng.standard_normal((n, 3, 3)) * 0.3 + np.eye(3) * rng.uniform(0.5, 2, size=(n, 1, 1))


def test_curvilinear_route_equals_cartesian_form():
    rng = np.random.default_rng(11)
    J = _random_J(rng, 50)
    for lam, mu in [(0.7, 0.4), (1.5, 0.1)]:
        A = macro_field(J, lam, mu)
        B = cartesian_field(J, lam, mu)
        scale = np.abs(B).max()
        np.testing.assert_allclose(A, B, atol=1e-13 * scale)


def test_field_symmetry_eq38():
    rng = np.random.default_rng(12)
    A = macro_field(_random_J(rng, 20), 0.9, 0.3)
    # A_ij = A_ji^T
    np.testing.assert_allclose(A, A.transpose(0, 2, 1, 4, 3), atol=1e-14 * np.abs(A).max())


def test_field_is_the_elastic_energy_density():
    """sum_ij u_,i^T A_ij v_,j equals det J (lam div u div v + 2 mu eps(u):eps(v)) in physical coordinates."""
    rng = np.random.default_rng(13)
    lam, mu = 0.8, 0.35
    J = _random_J(rng, 10)
    A = macro_field(J, lam, mu)
    for s in range(len(J)):
        du = rng.standard_normal((3, 3))   # du[i] = u_{,xi_i} (a 3-vector)
        dv = rng.standard_normal((3, 3))
        lhs = np.einsum("ia,ijab,jb->", du, A[s], dv)
        F = np.linalg.inv(J[s])
        Gu = np.einsum("ia,im->am", du, F)  # physical gradient d u_a / d x_m
        Gv = np.einsum("ia,im->am", dv, F)
        eu, ev = 0.5 * (Gu + Gu.T), 0.5 * (Gv + Gv.T)
        rhs = np.linalg.det(J[s]) * (lam * np.trace(Gu) * np.trace(Gv) + 2 * mu * np.sum(eu * ev))
        assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("q,n_fit", [(0, 1), (1, 2), (2, 3), (3, 4), (2, 5)])
def test_projection_reproduces_polynomials(q, n_fit):
    rng = np.random.default_rng(q + 10 * n_fit)
    d = rng.standard_normal(((q + 1) ** 3, 4))
    pts, _ = projection.fit_points(n_fit)
    f = projection.bernstein3(q, pts) @ d
    P = projection.projection_operator(q, n_fit)
    np.testing.assert_allclose(P @ f, d, atol=1e-12)


@pytest.mark.parametrize("q", [1, 2, 3])
def test_projection_with_q_plus_1_points_interpolates(q):
    rng = np.random.default_rng(q)
    pts, _ = projection.fit_points(q + 1)
    f = rng.standard_normal((len(pts), 2))
    P = projection.projection_operator(q, q + 1)
    np.testing.assert_allclose(projection.bernstein3(q, pts) @ (P @ f), f, atol=1e-12)


def test_bernstein3_ordering():
    q = 2
    x = np.array([[0.1, 0.5, 0.9]])
    N = projection.bernstein3(q, x)[0]
    B = [bernstein(q, x[:, k])[0] for k in range(3)]
    for c3 in range(3):
        for c2 in range(3):
            for c1 in range(3):
                assert N[c1 + 3 * (c2 + 3 * c3)] == pytest.approx(B[0][c1] * B[1][c2] * B[2][c3], rel=1e-15)


def test_identity_and_affine_maps():
    sp = W.identity_spline((2, 3, 2), (2, 3, 1))
    pts = np.random.default_rng(0).uniform(0, 1, size=(20, 3))
    X, J = geometry.eval_volume_points(sp.degree, sp.knots, sp.ctrl, pts)
    np.testing.assert_allclose(X, pts, atol=1e-14)
    np.testing.assert_allclose(J, np.broadcast_to(np.eye(3), J.shape), atol=1e-13)
    A = np.array([[1.0, 0.2, 0], [0, 1.3, 0.1], [0.2, 0, 0.8]])
    b = np.array([1.0, 2.0, 3.0])
    sp = W.affine_macro((3, 2, 2), (2, 2, 3), A, b)
    X, J = geometry.eval_volume_points(sp.degree, sp.knots, sp.ctrl, pts)
    np.testing.assert_allclose(X, pts @ A.T + b, atol=1e-13)
    np.testing.assert_allclose(J, np.broadcast_to(A, J.shape), atol=1e-12)


def test_tile_gluing_numbering():
    w = W.make("cfg1")
    nx, ny, nz = w.tile.n_ctrl
    G0 = geometry.tile_global_indices(w, 0).reshape(nz, ny, nx)
    G1 = geometry.tile_global_indices(w, 1).reshape(nz, ny, nx)   # +x neighbour
    np.testing.assert_array_equal(G0[:, :, -1], G1[:, :, 0])
    G2 = geometry.tile_global_indices(w, 2).reshape(nz, ny, nx)   # +y neighbour
    np.testing.assert_array_equal(G0[:, -1, :], G2[:, 0, :])
