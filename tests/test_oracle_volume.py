"""Pins for the volume V^pi (eq. (14)-(19), (25)-(26)) and its sensitivity (eq. (66)-(67)) of the oracle."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import volume

A = np.array([[1.3, 0.2, -0.1], [0.1, 0.8, 0.15], [-0.05, 0.1, 1.1]])


def _curved_trilinear(seed=4):
    """A degree-1 macro map with perturbed interior control points (det J_M > 0.17 everywhere):
    |det J_M| is a polynomial of degree 3 p_M - 1 = 2 per direction on each knot span (eq. (22)),
    reproduced by q = 2."""
    m = W.affine_macro((1, 1, 1), (3, 3, 3), A, np.array([0.5, -1.0, 2.0]))
    rng = np.random.default_rng(seed)
    ctrl = m.ctrl.copy()
    ctrl[1:-1, 1:-1, 1:-1] += 0.045 * rng.standard_normal(ctrl[1:-1, 1:-1, 1:-1].shape)
    return dataclasses.replace(m, ctrl=ctrl)


def _workload(macro, q, tiles=(2, 3, 2), tile=None, n_fit=None, box_mode=1):
    tile = W.make("cfg1").tile if tile is None else tile
    return W.Workload("vol", macro, tile, tiles, box_mode, q, q + 1 if n_fit is None else n_fit, 3)


def test_table_partition_of_unity_and_q0_fold():
    """sum_C t^h[C] = int |det J_T| = 1 (the tile maps onto the unit cube; sum_C N_C = 1);
    at q = 0 the adjoint field is the constant volume fraction t_pi = t^h = 1 (eq. (67))."""
    tile = W.make("cfg1").tile
    for q in (1, 2, 3):
        assert volume.volume_table(tile, q, 8).sum() == pytest.approx(1.0, abs=1e-13)
    t0 = volume.volume_table(tile, 0, 8)
    np.testing.assert_allclose(volume.folded_table(0, t0), [1.0], atol=1e-13)
    # the mass matrix of eq. (24) in one direction: int B_a B_b = C(q,a) C(q,b) / ((2q+1) C(2q,a+b))
    from math import comb
    q = 3
    M1 = np.array([[comb(q, a) * comb(q, b) / ((2 * q + 1) * comb(2 * q, a + b)) for b in range(q + 1)]
                   for a in range(q + 1)])
    np.testing.assert_allclose(volume.mass_matrix(q), np.kron(np.kron(M1, M1), M1), rtol=1e-13)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_affine_volume_is_det_A(q):
    """Affine M: |det J_M| is constant, V^pi = V. = |det A| (the macro parameter domain is the
    unit cube), and each tile's volume is |det A| times its box volume."""
    w = _workload(W.affine_macro((2, 2, 2), (2, 2, 2), A, np.zeros(3)), q)
    t_h = volume.volume_table(w.tile, q, 8)
    assert volume.volume(w, t_h) == pytest.approx(abs(np.linalg.det(A)), rel=1e-12)
    assert volume.volume_standard(w, 8) == pytest.approx(abs(np.linalg.det(A)), rel=1e-12)
    v = volume.tile_volumes(w, t_h)
    np.testing.assert_allclose(v, abs(np.linalg.det(A)) / w.n_tiles, rtol=1e-12)


def test_exact_projection_matches_full_quadrature_and_fold():
    """When q reaches the degree of |det J_M| the projection is exact, so V^pi equals the full
    quadrature of eq. (14) with the same micro Gauss points; the folded table (eq. (25)) gives
    the same volume.  Tiles are the macro knot spans, where |det J_M| is one polynomial."""
    w = _workload(_curved_trilinear(), 2, tiles=(3, 3, 3), box_mode=0)
    t_h = volume.volume_table(w.tile, 2, 3)
    v_pi = volume.volume(w, t_h)
    v_std = volume.volume_standard(w, 3)
    assert v_pi == pytest.approx(v_std, rel=1e-13)
    assert volume.volume_folded(w, volume.folded_table(2, t_h)) == pytest.approx(v_pi, rel=1e-13)
    # a lower degree does not reproduce it (the L2 projection keeps the mean, so the gap is small)
    w1 = dataclasses.replace(w, q=1, n_fit=2)
    assert abs(volume.volume(w1, volume.volume_table(w.tile, 1, 3)) - v_std) > 1e-10 * v_std


def test_curved_volume_error_decreases_with_q():
    w0 = W.make("cfg1")
    v_std = volume.volume_standard(w0)
    errs = []
    for q in (0, 1, 2, 3, 4):
        w = dataclasses.replace(w0, q=q, n_fit=q + 1)
        errs.append(abs(volume.volume(w, volume.volume_table(w.tile, q, w.n_gauss)) - v_std) / v_std)
    assert all(b < a for a, b in zip(errs[:-1], errs[1:])), errs


@pytest.mark.parametrize("name,q", [("trilinear", 2), ("cfg1", 2), ("cfg1", 0)])
def test_gradient_against_central_differences(name, q):
    """eq. (66)-(67) equals the derivative of the discrete V^pi (central differences)."""
    if name == "trilinear":
        w = _workload(_curved_trilinear(), q, tiles=(2, 2, 2))
    else:
        w = dataclasses.replace(W.make("cfg1"), q=q, n_fit=q + 1)
    t_h = volume.volume_table(w.tile, q, w.n_gauss)
    g = volume.volume_grad(w, volume.folded_table(q, t_h))
    rng = np.random.default_rng(8)
    nz, ny, nx = w.macro.ctrl.shape[:3]
    picks = [(0, 0, 0, 0), (nz - 1, ny - 1, nx - 1, 2)] + [
        (rng.integers(nz), rng.integers(ny), rng.integers(nx), rng.integers(3)) for _ in range(4)]
    eps = 1e-6
    for (k, j, i, c) in picks:
        vals = []
        for sgn in (1, -1):
            ctrl = w.macro.ctrl.copy()
            ctrl[k, j, i, c] += sgn * eps
            ws = dataclasses.replace(w, macro=dataclasses.replace(w.macro, ctrl=ctrl))
            vals.append(volume.volume(ws, t_h))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert g[k, j, i, c] == pytest.approx(fd, rel=1e-6, abs=1e-9), (k, j, i, c)
