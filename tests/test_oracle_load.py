"""Pins for the load vector f^pi (eq. (39)-(41), (44)-(45), (53)-(55)) of the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import load

BODY = np.array([0.3, -1.2, 0.7])
TRACTION = np.array([[1.0, 0.0, 0.5], [0.0, -2.0, 1.0], [0.4, 0.1, 0.0],
                     [-0.3, 0.2, 0.9], [0.0, 0.0, -1.5], [2.0, 1.0, 0.3]])   # faces 2 d + side


def _affine(q, tiles=(2, 3, 2), box_mode=1, tile=None):
    A = np.array([[1.3, 0.2, -0.1], [0.1, 0.8, 0.15], [-0.05, 0.1, 1.1]])
    b = np.array([0.5, -1.0, 2.0])
    macro = W.affine_macro((2, 2, 2), (2, 2, 2), A, b)
    tile = W.make("cfg1").tile if tile is None else tile
    return W.Workload("affine", macro, tile, tiles, box_mode, q, q + 1, 3), A


@pytest.mark.parametrize("q", [1, 2, 3])
def test_table_closed_forms(q):
    """sum_A F[A,C,0] = int_[0,1]^3 N_C = (q+1)^-3 (partition of unity of R_A, T^r onto the cube);
    sum_A F[A,C,1+f] = (q+1)^-2 for C in I_f and 0 otherwise (N_C vanishes on face f off I_f)."""
    q1 = q + 1
    # identity tile: N_C(T(theta)) det J_T is a polynomial the Gauss rule integrates exactly
    Fi = load.load_table(W.identity_spline((2, 2, 2), (2, 2, 2)), q, 3)
    np.testing.assert_allclose(Fi[:, :, 0].sum(axis=0), q1 ** -3.0, rtol=1e-13)
    # pulled tile: with 8 points per direction the rule resolves the curved tile map as well
    tile = W.make("cfg1").tile
    np.testing.assert_allclose(load.load_table(tile, q, 8)[:, :, 0].sum(axis=0), q1 ** -3.0, rtol=1e-13)
    F = load.load_table(tile, q, 3)
    for f in range(6):
        s = F[:, :, 1 + f].sum(axis=0)
        I = load.face_index_set(q, f)
        assert len(I) == q1 * q1
        np.testing.assert_allclose(s[I], q1 ** -2.0, rtol=1e-13)
        mask = np.ones(q1 ** 3, bool)
        mask[I] = False
        assert np.abs(s[mask]).max() < 1e-15
    # only the face's own control points carry face integrals
    n = tile.n_ctrl
    for f in range(6):
        d, side, _, _ = load.face_axes(f)
        for A in range(int(np.prod(n))):
            idx = (A % n[0], (A // n[0]) % n[1], A // (n[0] * n[1]))
            if idx[d] != (n[d] - 1 if side else 0):
                assert np.abs(F[A, :, 1 + f]).max() == 0.0


@pytest.mark.parametrize("q", [0, 1, 2])
def test_affine_map_equals_quadrature_and_totals(q):
    """Affine M: |det J| and the face area elements are constant, the projections are exact, and
    f^pi equals the Gauss-quadrature f^bullet to rounding; both carry the total force
    b |det A| + sum_f t_f |A e_u x A e_v| (partition of unity)."""
    w, A = _affine(q)
    F = load.load_table(w.tile, q, 3)
    fpi = load.assemble_load(w, F, BODY, TRACTION)
    fstd = load.standard_load(w, BODY, TRACTION)
    assert np.linalg.norm(fpi - fstd) <= 1e-13 * np.linalg.norm(fstd)
    total = BODY * abs(np.linalg.det(A))
    for f in range(6):
        _, _, u, v = load.face_axes(f)
        total = total + TRACTION[f] * np.linalg.norm(np.cross(A[:, u], A[:, v]))
    for a in range(3):
        assert fpi[a::3].sum() == pytest.approx(total[a], rel=1e-12, abs=1e-12)
        assert fstd[a::3].sum() == pytest.approx(total[a], rel=1e-12, abs=1e-12)


def test_faces_only_on_the_macro_boundary():
    """Interior tiles get no traction; a single face's traction lands on that face's points only."""
    w, A = _affine(1)
    F = load.load_table(w.tile, 1, 3)
    tr = np.zeros((6, 3))
    tr[3] = [0.0, 1.0, 0.0]                              # face xi_2 = 1
    f = load.assemble_load(w, F, np.zeros(3), tr)
    GX, GY, GZ = (w.tiles[0] * 3 + 1, w.tiles[1] * 3 + 1, w.tiles[2] * 3 + 1)
    fy = f[1::3].reshape(GZ, GY, GX)
    assert np.abs(fy[:, :-1, :]).max() == 0.0
    assert fy[:, -1, :].sum() == pytest.approx(np.linalg.norm(np.cross(A[:, 0], A[:, 2])), rel=1e-12)
    assert np.abs(f[0::3]).max() == 0.0 and np.abs(f[2::3]).max() == 0.0


def test_curved_map_vector_error_decreases_with_q():
    """Curved macro map (cfg1): E_vec = |f^bullet - f^pi| / |f^bullet| (eq. (63)) is small and
    decreases with the projection degree; the totals agree to the same order."""
    w0 = W.make("cfg1")
    fstd = load.standard_load(w0, BODY, TRACTION)
    errs = []
    for q in (1, 2, 3, 4):
        w = W.Workload("q", w0.macro, w0.tile, w0.tiles, 0, q, q + 1, 3)
        F = load.load_table(w.tile, q, 3)
        fpi = load.assemble_load(w, F, BODY, TRACTION)
        errs.append(np.linalg.norm(fpi - fstd) / np.linalg.norm(fstd))
    assert all(b < a for a, b in zip(errs[:-1], errs[1:])), errs
    assert errs[1] < 1e-3, errs
