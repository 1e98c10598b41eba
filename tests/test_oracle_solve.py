"""Pins for the solved system K^pi u = f^pi (eq. (30), (50), (53)) of the oracle."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import assembly, geometry, load, projection, solve, tables


def _system(w, traction):
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    blocks = assembly.tile_blocks(T, projection.all_coefficients(w))
    rp, ci, vals = assembly.assemble_csr(w, pairs, blocks)
    f = load.assemble_load(w, load.load_table(w.tile, w.q, w.n_gauss), np.zeros(3), traction)
    return rp, ci, vals, f


@pytest.mark.parametrize("tile", ["identity", "cfg1"])
def test_clamped_bar_patch_test(tile):
    """A box (affine macro map), clamped on xi_3 = 0, pulled by a uniform traction t e_3 on
    xi_3 = 1, with nu = 0: the exact displacement u = (0, 0, t z / E) is linear, hence in the
    discrete space of the composed (isoparametric) map, and the Galerkin solution reproduces it at
    every control point, also through a curved tile parametrisation.  The lateral faces are free:
    with nu = 0 the uniaxial stress needs no lateral contraction."""
    A = np.diag([0.7, 0.9, 2.0])
    macro = W.affine_macro((1, 1, 1), (1, 1, 1), A, np.array([0.1, -0.2, 0.3]))
    t_tile = W.identity_spline((2, 2, 2), (2, 2, 2)) if tile == "identity" else W.make("cfg1").tile
    w = W.Workload("bar", macro, t_tile, (2, 2, 3), 1, 1, 2, 3, E=3.0, nu=0.0)
    traction = np.zeros((6, 3))
    traction[5] = [0.0, 0.0, 0.6]
    rp, ci, vals, f = _system(w, traction)
    fixed = solve.face_dofs(w, 4)
    u = solve.dirichlet_solve(rp, ci, vals, f, fixed)
    X = geometry.composed_control_points(w)
    z = X[:, 2] - 0.3                               # distance from the clamped face
    exact = np.zeros_like(u)
    exact[2::3] = 0.6 * z / 3.0
    assert np.abs(u - exact).max() <= 1e-12 * np.abs(exact).max()


def test_face_dofs_and_residual():
    """Face masks pick one layer of control points; the solution satisfies the free equations and
    vanishes on the clamped dofs; a rigid translation of the clamped face is not in the kernel."""
    w = W.make("cfg1")
    G = geometry.global_grid(w)
    for face in range(6):
        m = solve.face_dofs(w, face)
        d = face // 2
        assert m.sum() == 3 * np.prod(G) // G[d]
    traction = np.zeros((6, 3))
    traction[1] = [0.2, -0.1, 0.4]
    rp, ci, vals, f = _system(w, traction)
    fixed = solve.face_dofs(w, 0)
    u = solve.dirichlet_solve(rp, ci, vals, f, fixed)
    assert np.abs(u[fixed]).max() == 0.0
    r = assembly.spmv(rp, ci, vals, u) - f
    assert np.linalg.norm(r[~fixed]) <= 1e-10 * np.linalg.norm(f)
    assert np.linalg.norm(u) > 0
