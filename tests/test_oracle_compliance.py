"""Pins for the oracle's compliance sensitivity with a load that moves with the geometry
(Section 4.1.2, eq. (68)-(73); the external work of eq. (69) differentiated through the load
projections of eq. (40)-(41), (44)-(45)).

c(m) = f(m)^T K(m)^-1 f(m) with f = f^pi(m) the library's load vector (its body term carries
|det J| and its face term the face area element, both of which move with the macro control points).
With u = K^-1 f: dc/dm = 2 u . df/dm - u^T (dK/dm) u.  The pins are central differences of c with
the load and the matrix re-assembled and the system re-solved for every perturbation, and of u.f
for a fixed u; none of them uses the adjoint formulas being pinned.
"""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, assembly, geometry, load, projection, solve, tables


def _perturbed(w, idx, h):
    m = replace(w.macro, ctrl=w.macro.ctrl.copy())
    m.ctrl[idx] += h
    return replace(w, macro=m)


BODY = np.array([0.0, 0.0, -0.5])


def _traction():
    t = np.zeros((6, 3))
    t[1] = [0.0, 0.0, -1.0]      # uniform traction on xi_1 = 1
    return t


@pytest.mark.parametrize("name,kw", [("cfg4", {"n_boxes": 2}), ("nurbs_torus", {"n_boxes": 2})])
def test_load_gradient_vs_central_fd(name, kw):
    w = W.make(name, **kw)
    trac = _traction()
    trac[4] = [0.3, -0.2, 0.1]   # and a traction on xi_3 = 0
    F = load.load_table(w.tile, w.q, w.n_gauss)
    u = W.random_displacement(geometry.n_global_dofs(w), 17)
    g = load.grad_uf(w, F, BODY, trac, u)
    assert np.abs(g).max() > 0
    rng = np.random.default_rng(4)
    nz, ny, nx, _ = w.macro.ctrl.shape
    h = 1e-6
    for _ in range(6):
        idx = (int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx)), int(rng.integers(3)))
        fd = (load.uf(_perturbed(w, idx, h), F, BODY, trac, u) - load.uf(_perturbed(w, idx, -h), F, BODY, trac, u)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(g).max())


def test_load_gradient_zero_without_loads():
    w = W.make("cfg4", n_boxes=2)
    F = load.load_table(w.tile, w.q, w.n_gauss)
    u = W.random_displacement(geometry.n_global_dofs(w), 3)
    assert np.all(load.grad_uf(w, F, np.zeros(3), np.zeros((6, 3)), u) == 0.0)


def test_load_gradient_translation_and_affine_body():
    """A rigid translation of the macro net changes no |det J| and no face area, so the gradient
    summed over all control points (the derivative along a translation) vanishes."""
    w = W.make("cfg4", n_boxes=2)
    F = load.load_table(w.tile, w.q, w.n_gauss)
    u = W.random_displacement(geometry.n_global_dofs(w), 5)
    g = load.grad_uf(w, F, BODY, _traction(), u)
    assert np.abs(g.reshape(-1, 3).sum(axis=0)).max() < 1e-12 * np.abs(g).max() * g.size


@pytest.fixture(scope="module")
def compliance_4():
    """The differentiation workload at 4^3 boxes: clamp xi_1 = 0, traction (0, 0, -1) on xi_1 = 1."""
    w = W.make("cfg4", n_boxes=4)
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    F = load.load_table(w.tile, w.q, w.n_gauss)
    fixed = solve.face_dofs(w, 0)
    return w, pairs, T, F, fixed


def _solve(wk, pairs, T, f, fixed):
    rp, ci, v = assembly.assemble_csr(wk, pairs, assembly.tile_blocks(T, projection.all_coefficients(wk)))
    return solve.dirichlet_solve(rp, ci, v, f, fixed)


def _fd_points(w, n):
    rng = np.random.default_rng(12)
    nz, ny, nx, _ = w.macro.ctrl.shape
    return [(int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx)), int(rng.integers(3)))
            for _ in range(n)]


def test_compliance_moving_load_direct_solve(compliance_4):
    w, pairs, T, F, fixed = compliance_4
    trac = _traction()

    def c_of(wk):
        f = load.assemble_load(wk, F, BODY, trac)
        return f @ _solve(wk, pairs, T, f, fixed)

    f0 = load.assemble_load(w, F, BODY, trac)
    u = _solve(w, pairs, T, f0, fixed)
    g_load = load.grad_uf(w, F, BODY, trac, u)
    grad = 2.0 * g_load - adjoint.grad_uKu(w, T, pairs, u)
    h = 1e-6
    scale = np.abs(grad).max()
    for idx in _fd_points(w, 3):
        fd = (c_of(_perturbed(w, idx, h)) - c_of(_perturbed(w, idx, -h))) / (2 * h)
        assert grad[idx] == pytest.approx(fd, rel=1e-5, abs=1e-7 * scale)
    # the load term is not negligible for this load: dropping it misses the derivative
    assert np.abs(2.0 * g_load).max() > 1e-2 * scale


def test_compliance_frozen_load_direct_solve(compliance_4):
    """The load computed once at the initial geometry and kept: dc/dm = -u^T (dK/dm) u."""
    w, pairs, T, F, fixed = compliance_4
    f = load.assemble_load(w, F, BODY, _traction())
    u = _solve(w, pairs, T, f, fixed)
    grad = -adjoint.grad_uKu(w, T, pairs, u)
    h = 1e-6
    scale = np.abs(grad).max()
    for idx in _fd_points(w, 3):
        fd = (f @ _solve(_perturbed(w, idx, h), pairs, T, f, fixed)
              - f @ _solve(_perturbed(w, idx, -h), pairs, T, f, fixed)) / (2 * h)
        assert grad[idx] == pytest.approx(fd, rel=1e-5, abs=1e-7 * scale)
