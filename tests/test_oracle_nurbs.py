"""Pins for NURBS macro maps (rational fields, Section 2.1 and the exact torus of Section 3.3.4)
in the oracle."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import adaptive, geometry, volume


def test_unit_weights_reduce_to_the_bspline():
    w = W.make("cfg1")
    x = np.linspace(0.0, 1.0, 4)
    X0, J0 = geometry.eval_volume_grid(w.macro.degree, w.macro.knots, w.macro.ctrl, x, x, x)
    ones = np.ones(w.macro.ctrl.shape[:3])
    X1, J1 = geometry.eval_volume_grid(w.macro.degree, w.macro.knots, w.macro.ctrl, x, x, x, weights=ones)
    np.testing.assert_allclose(X1, X0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(J1, J0, rtol=0, atol=1e-13)


def test_torus_points_and_jacobian_are_exact():
    """Every point of the NURBS quarter torus sits at tube distance rho(y) from the centre circle
    of radius R, at tube angle and revolution angle that the map's derivatives confirm: the
    Jacobian against a central difference of the rational map itself."""
    R, r1, r2 = 2.0, 0.5, 1.0
    m = W.nurbs_quarter_torus(R, r1, r2)
    rng = np.random.default_rng(3)
    pts = rng.random((40, 3))
    X, J = geometry.eval_volume_points(m.degree, m.knots, m.ctrl, pts, weights=m.weights)
    d = np.hypot(X[:, 0], X[:, 1])
    rho = np.hypot(d - R, X[:, 2])
    np.testing.assert_allclose(rho, r1 + (r2 - r1) * pts[:, 1], rtol=1e-14)
    eps = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = eps
        Xp, _ = geometry.eval_volume_points(m.degree, m.knots, m.ctrl, pts + e, weights=m.weights)
        Xm, _ = geometry.eval_volume_points(m.degree, m.knots, m.ctrl, pts - e, weights=m.weights)
        np.testing.assert_allclose(J[:, :, k], (Xp - Xm) / (2 * eps), rtol=1e-8, atol=1e-9)
    assert np.all(np.linalg.det(J) > 0)


def test_torus_volume_closed_form():
    """Full quadrature of eq. (14) over the microstructured torus (tiles fill the macro domain)
    against the exact volume (pi/2) (R (r2^2 - r1^2) pi/4 + (r2^3 - r1^3) / 3); the interpolation-
    and-lookup volume converges to it with q (the rational |det J_M| is not a polynomial)."""
    R, r1, r2 = 2.0, 0.5, 1.0
    exact = 0.5 * np.pi * (R * (r2 ** 2 - r1 ** 2) * np.pi / 4 + (r2 ** 3 - r1 ** 3) / 3)
    w = W.make("nurbs_torus", n_boxes=2)
    assert volume.volume_standard(w, 8) == pytest.approx(exact, rel=1e-11)
    errs = []
    for q in (1, 2, 3, 4):
        wq = dataclasses.replace(w, q=q, n_fit=q + 1)
        errs.append(abs(volume.volume(wq, volume.volume_table(w.tile, q, 8)) - exact) / exact)
    assert all(b < a for a, b in zip(errs[:-1], errs[1:])), errs
    assert errs[-1] < 1e-7
    # the projection error of the macro field of a rational map falls with q as well
    e = [adaptive.eproj(w, q) for q in (2, 3, 4)]
    assert e[0] > e[1] > e[2] > 0


def test_nurbs_gradients_against_differences():
    """Volume and compliance gradients of the rational torus map (weights fixed) against central
    differences of the oracle's own V^pi and u^T K^pi u."""
    from oracle import adjoint, tables
    w = W.make("nurbs_torus", n_boxes=2)
    t_h = volume.volume_table(w.tile, w.q, w.n_gauss)
    gv = volume.volume_grad(w, volume.folded_table(w.q, t_h))
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    n = 3 * int(np.prod([w.tiles[k] * (w.tile.n_ctrl[k] - 1) + 1 for k in range(3)]))
    u = W.random_displacement(n, 5) * 0.1
    gc = adjoint.grad_uKu(w, T, pairs, u)
    eps = 1e-6
    for idx in [(1, 1, 1, 0), (0, 2, 1, 2), (2, 0, 2, 1)]:
        vv, cc = [], []
        for sgn in (1, -1):
            c = w.macro.ctrl.copy()
            c[idx] += sgn * eps
            ws = dataclasses.replace(w, macro=dataclasses.replace(w.macro, ctrl=c))
            vv.append(volume.volume(ws, t_h))
            cc.append(adjoint.uKu(ws, T, pairs, u))
        assert gv[idx] == pytest.approx((vv[0] - vv[1]) / (2 * eps), rel=1e-6, abs=1e-9)
        assert gc[idx] == pytest.approx((cc[0] - cc[1]) / (2 * eps), rel=1e-6, abs=1e-9)
