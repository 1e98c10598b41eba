"""Pins for the oracle's sensitivity (Section 4.1.2) and learned-table (POD + MLP) parts."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import adjoint, assembly, geometry, learned, projection, tables


def _perturbed(w, idx, h):
    m = w.macro.copy()
    m.ctrl[idx] += h
    return W.Workload(w.name, m, w.tile, w.tiles, w.box_mode, w.q, w.n_fit, w.n_gauss, w.E, w.nu)


@pytest.fixture(scope="module")
def small_cfg4():
    w = W.make("cfg4", n_boxes=3)
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    u = W.random_displacement(geometry.n_global_dofs(w), 7)
    return w, pairs, T, u


def test_uKu_gradient_vs_central_fd(small_cfg4):
    w, pairs, T, u = small_cfg4
    g = adjoint.grad_uKu(w, T, pairs, u)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(6):
        k = tuple(int(v) for v in rng.integers(0, 8, size=3))
        c = int(rng.integers(0, 3))
        idx = (k[2], k[1], k[0], c)
        tl = adjoint.tiles_touching(w, k)
        fd = (adjoint.uKu(_perturbed(w, idx, h), T, pairs, u, tl)
              - adjoint.uKu(_perturbed(w, idx, -h), T, pairs, u, tl)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(g).max())


def test_uKu_equals_quadratic_form(small_cfg4):
    w, pairs, T, u = small_cfg4
    blocks = assembly.tile_blocks(T, projection.all_coefficients(w))
    K = assembly.to_scipy(*assembly.assemble_csr(w, pairs, blocks))
    assert adjoint.uKu(w, T, pairs, u) == pytest.approx(u @ (K @ u), rel=1e-12)


def test_compliance_gradient_with_direct_solve():
    """c = f^T K^-1 f with a fixed load: dc/dm = -d(u^T K u)/dm |_u, u = K^-1 f (eq. (69), load term
    dropped because the load does not depend on m)."""
    w = W.make("cfg4", n_boxes=2)
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    GX, GY, GZ = geometry.global_grid(w)
    g = np.arange(GX * GY * GZ)
    free = (3 * g[(g % GX) != 0][:, None] + np.arange(3)).ravel()
    f = np.zeros(geometry.n_global_dofs(w))
    rng = np.random.default_rng(9)
    f[free] = rng.standard_normal(len(free)) * 0.01

    def solve(wk):
        blocks = assembly.tile_blocks(T, projection.all_coefficients(wk))
        K = assembly.to_scipy(*assembly.assemble_csr(wk, pairs, blocks)).tocsc()
        u = np.zeros_like(f)
        u[free] = spla.spsolve(K[free][:, free], f[free])
        return u

    u = solve(w)
    grad = -adjoint.grad_uKu(w, T, pairs, u)
    h = 1e-6
    for idx in [(3, 2, 5, 0), (1, 4, 4, 2), (6, 6, 1, 1)]:
        cp = f @ solve(_perturbed(w, idx, h))
        cm = f @ solve(_perturbed(w, idx, -h))
        fd = (cp - cm) / (2 * h)
        assert grad[idx] == pytest.approx(fd, rel=1e-5, abs=1e-8 * np.abs(grad).max())


def test_pod_orthonormal_and_eckart_young():
    rng = np.random.default_rng(21)
    X = rng.standard_normal((40, 7)) @ rng.standard_normal((7, 300)) + 0.01 * rng.standard_normal((40, 300))
    mean, basis, sigma = learned.pod(X, 5)
    np.testing.assert_allclose(basis.T @ basis, np.eye(5), atol=1e-12)
    Xc = X - mean
    Xr = (Xc @ basis) @ basis.T
    res = np.sum((Xc - Xr) ** 2)
    assert res == pytest.approx(np.sum(sigma[5:] ** 2), rel=1e-9)
    sv = np.linalg.svd(Xc, compute_uv=False)[:-1]   # centring removes one rank
    np.testing.assert_allclose(sigma[:len(sv)], sv, rtol=1e-9, atol=1e-9 * sv[0])


def test_mlp_backward_vs_fd():
    params = learned.init_mlp([4, 16, 16, 8], seed=3)
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, size=(10, 4))
    target = rng.standard_normal((10, 8))
    L, grads = learned.loss_and_grads(params, x, target)
    h = 1e-6
    for li, P in enumerate(params):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in P.shape)
            P[idx] += h
            lp, _ = learned.loss_and_grads(params, x, target)
            P[idx] -= 2 * h
            lm, _ = learned.loss_and_grads(params, x, target)
            P[idx] += h
            assert grads[li][idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-10)


def test_gelu_grad_vs_fd():
    z = np.linspace(-4, 4, 33)
    h = 1e-6
    np.testing.assert_allclose(learned.gelu_grad(z), (learned.gelu(z + h) - learned.gelu(z - h)) / (2 * h), atol=1e-9)


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -0.1, 2.0])
    m = np.zeros(3); v = np.zeros(3)
    learned.adam_update(p, g, m, v, step=1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p, [0.99, -1.99, 2.99], atol=1e-15)
