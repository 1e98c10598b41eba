"""Pins for the whole interpolation-and-lookup operator K^pi (eq. (50), (58)) and its global assembly."""
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import assembly, geometry, projection, standard, tables


def _fast_blocks(w, pairs=None):
    pairs = tables.pair_set(w.tile) if pairs is None else pairs
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    return pairs, assembly.tile_blocks(T, projection.all_coefficients(w))


def _affine_workload(q, tile=None, box_mode=0, tiles=(2, 2, 2)):
    A = np.array([[1.3, 0.2, -0.1], [0.1, 0.8, 0.15], [-0.05, 0.1, 1.1]])
    b = np.array([0.5, -1.0, 2.0])
    macro = W.affine_macro((2, 2, 2), (2, 2, 2), A, b)
    tile = W.make("cfg1").tile if tile is None else tile
    return W.Workload("affine", macro, tile, tiles, box_mode, q, q + 1, 3)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_affine_macro_matches_standard_gauss(q):
    """Affine M: A is constant, the projection is exact and K^pi equals K^bullet to rounding."""
    w = _affine_workload(q)
    pairs, blocks = _fast_blocks(w)
    for t in range(w.n_tiles):
        ref = standard.tile_block_standard(w, t, pairs)
        assert np.linalg.norm(blocks[t] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_affine_cubic_tile_uniform_boxes():
    tile = W.make("cfg2").tile
    w = _affine_workload(1, tile=tile, box_mode=1, tiles=(1, 1, 2))
    pairs, blocks = _fast_blocks(w)
    ref = standard.tile_block_standard(w, 1, pairs)
    assert np.linalg.norm(blocks[1] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_curved_emat_decreases_with_q():
    """Section 3.3.1: every error decreases as the projection degree grows."""
    w0 = W.make("cfg1")
    pairs = tables.pair_set(w0.tile)
    ref = np.stack([standard.tile_block_standard(w0, t, pairs) for t in range(w0.n_tiles)])
    errs = []
    for q in range(7):
        w = W.Workload("q", w0.macro, w0.tile, w0.tiles, 0, q, q + 1, 3)
        _, blocks = _fast_blocks(w, pairs)
        errs.append(np.linalg.norm(blocks - ref) / np.linalg.norm(ref))
    assert all(b < a for a, b in zip(errs[:-1], errs[1:])), errs
    assert errs[-1] < 1e-6


@pytest.fixture(scope="module")
def cfg1_global():
    w = W.make("cfg1")
    pairs, blocks = _fast_blocks(w)
    rp, ci, v = assembly.assemble_csr(w, pairs, blocks)
    return w, pairs, blocks, assembly.to_scipy(rp, ci, v)


def test_translations_in_kernel(cfg1_global):
    w, pairs, blocks, K = cfg1_global
    n = K.shape[0]
    scale = abs(K).max()
    for a in range(3):
        t = np.zeros(n)
        t[a::3] = 1.0
        assert np.abs(K @ t).max() < 1e-13 * scale * 10


def test_rotations_in_kernel_only_for_affine_maps():
    w = _affine_workload(1)
    pairs, blocks = _fast_blocks(w)
    rp, ci, v = assembly.assemble_csr(w, pairs, blocks)
    K = assembly.to_scipy(rp, ci, v)
    X = geometry.composed_control_points(w)
    scale = abs(K).max() * np.abs(X).max()
    for axis in range(3):
        om = np.zeros(3)
        om[axis] = 1.0
        u = np.cross(om, X).ravel()
        assert np.abs(K @ u).max() < 1e-12 * scale
    # curved map: rotations leave a residual (the composed geometry is not in the discrete space)
    wc = W.make("cfg1")
    pairs, blocks = _fast_blocks(wc)
    rp, ci, v = assembly.assemble_csr(wc, pairs, blocks)
    Kc = assembly.to_scipy(rp, ci, v)
    u = np.cross(np.array([0, 0, 1.0]), geometry.composed_control_points(wc)).ravel()
    assert np.abs(Kc @ u).max() > 1e-8 * abs(Kc).max()


def test_patch_test_affine():
    """Linear displacement on an affine macro map: interior rows of K u vanish."""
    w = _affine_workload(2)
    pairs, blocks = _fast_blocks(w)
    rp, ci, v = assembly.assemble_csr(w, pairs, blocks)
    K = assembly.to_scipy(rp, ci, v)
    X = geometry.composed_control_points(w)
    H = np.array([[0.3, -0.1, 0.2], [0.05, 0.4, -0.2], [0.1, 0.2, -0.3]])
    u = (X @ H.T + np.array([0.1, 0.2, 0.3])).ravel()
    r = (K @ u).reshape(-1, 3)
    GX, GY, GZ = geometry.global_grid(w)
    g = np.arange(GX * GY * GZ)
    gx, gy, gz = g % GX, (g // GX) % GY, g // (GX * GY)
    interior = (gx > 0) & (gx < GX - 1) & (gy > 0) & (gy < GY - 1) & (gz > 0) & (gz < GZ - 1)
    assert np.abs(r[interior]).max() < 1e-12 * abs(K).max() * np.abs(u).max()
    assert np.abs(r[~interior]).max() > 1e-6


def test_clamped_stiffness_is_positive_definite(cfg1_global):
    w, pairs, blocks, K = cfg1_global
    GX, GY, GZ = geometry.global_grid(w)
    g = np.arange(GX * GY * GZ)
    free_pts = (g % GX) != 0
    free = (3 * g[free_pts][:, None] + np.arange(3)).ravel()
    Kf = K.toarray()[np.ix_(free, free)]
    scipy.linalg.cholesky(Kf)
    np.testing.assert_allclose(Kf, Kf.T, atol=0)


def test_csr_equals_dense_sum_of_tiles(cfg1_global):
    w, pairs, blocks, K = cfg1_global
    D = assembly.dense_global(w, pairs, blocks)
    np.testing.assert_allclose(K.toarray(), D, atol=1e-15 * np.abs(D).max())


def _nnz_closed_form(w):
    """Pattern size from 1-D global neighbour counts: nnz = 9 prod_k sum_g c_k(g)."""
    total = 9
    for k in range(3):
        n, p, T = w.tile.n_ctrl[k], w.tile.degree[k], w.tiles[k]
        NG = T * (n - 1) + 1
        cnt = 0
        for g in range(NG):
            nb = set()
            for t in range(T):
                lo = t * (n - 1)
                if lo <= g <= lo + n - 1:
                    nb |= {lo + j for j in range(n) if abs(j - (g - lo)) <= p}
            cnt += len(nb)
        total *= cnt
    return total


def test_pattern_size_closed_form(cfg1_global):
    w, pairs, blocks, K = cfg1_global
    assert K.nnz == _nnz_closed_form(w) == 177147


def test_sampled_rows_match_global(cfg1_global):
    w, pairs, blocks, K = cfg1_global
    rows = [0, 5, 77, 500, K.shape[0] - 1]
    got = assembly.csr_rows(w, pairs, lambda t: blocks[t], rows)
    for r in rows:
        cols, vals = got[r]
        sl = slice(K.indptr[r], K.indptr[r + 1])
        np.testing.assert_array_equal(cols, K.indices[sl])
        np.testing.assert_allclose(vals, K.data[sl], atol=1e-16 * abs(K).max(), rtol=1e-14)


def test_quadrature_convergence_single_tile():
    """Brute force on one tile: more Gauss points change K^bullet only at the quadrature-error level,
    and K^pi and K^bullet agree with the same rule up to the projection error."""
    w = W.make("cfg1")
    pairs = tables.pair_set(w.tile)
    k3 = standard.tile_block_standard(w, 3, pairs, n_g=3)
    k8 = standard.tile_block_standard(w, 3, pairs, n_g=8)
    assert np.linalg.norm(k8 - k3) / np.linalg.norm(k8) < 1e-3
    _, blocks = _fast_blocks(w, pairs)
    assert np.linalg.norm(blocks[3] - k3) / np.linalg.norm(k3) < 1e-3


def test_linop_equals_assembled_matrix(cfg1_global):
    """Eq. (74): the tile-by-tile product equals the assembled CSR matrix times u, and for an
    affine map the standard Gauss-quadrature matrix times u."""
    w, pairs, blocks, _ = cfg1_global
    rp, ci, vals = assembly.assemble_csr(w, pairs, blocks)
    u = W.random_displacement(geometry.n_global_dofs(w), 3)
    y = assembly.linop_apply(w, pairs, blocks, u)
    ref = assembly.spmv(rp, ci, vals, u)
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    wa = _affine_workload(2, tiles=(2, 1, 2), box_mode=1)
    pa, ba = _fast_blocks(wa)
    ua = W.random_displacement(geometry.n_global_dofs(wa), 4)
    ya = assembly.linop_apply(wa, pa, ba, ua)
    Kstd = np.zeros((geometry.n_global_dofs(wa),) * 2)
    for t in range(wa.n_tiles):
        d = geometry.tile_dofs(wa, t)
        Kstd[np.ix_(d, d)] += standard.tile_matrix_standard(wa, t)
    assert np.linalg.norm(ya - Kstd @ ua) <= 1e-12 * np.linalg.norm(Kstd @ ua)
