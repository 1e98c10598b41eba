"""Contraction and global sparse assembly (oracle, test infrastructure only).

Eq. (58): nzdata = mat[K] . mat[<A>]  -- done here one tile at a time with np.matmul:
  block^(t) = table @ Coef^(t),  shape (n_nz, 9), column 3 a + b, so that for (A, B) = pairs[p]
  K^(t)[(A,a), (B,b)] = block^(t)[p, 3a+b]  and by symmetry  K^(t)[(B,b), (A,a)] = the same value.
Step 4 of Section 3.2.4: scatter all tile blocks into one global matrix.  The
pattern is the brute-force set of all (row, col) touched by any tile (full
symmetric storage, sorted columns); values are summed over tiles in ascending
tile order.
"""
from __future__ import annotations

import numpy as np

from .geometry import n_global_dofs, tile_dofs, tile_global_indices


def tile_blocks(table: np.ndarray, coefs: np.ndarray) -> np.ndarray:
    """(T, n_nz, 9) stack of table @ Coef^(t)."""
    return np.matmul(table[None, :, :], coefs)


def tile_dense(pairs: np.ndarray, block: np.ndarray, nT: int) -> np.ndarray:
    """Dense (3 n_T, 3 n_T) tile stiffness from its upper-pair block."""
    K = np.zeros((3 * nT, 3 * nT))
    for p, (A, B) in enumerate(pairs):
        blk = block[p].reshape(3, 3)
        K[3 * A:3 * A + 3, 3 * B:3 * B + 3] = blk
        K[3 * B:3 * B + 3, 3 * A:3 * A + 3] = blk.T
    return K


def coo_entries(w, pairs: np.ndarray, blocks: np.ndarray, tiles=None):
    """All (row, col, value) contributions in ascending tile order (both triangles)."""
    tiles = range(w.n_tiles) if tiles is None else tiles
    rows, cols, vals = [], [], []
    ab = np.arange(9)
    a, b = ab // 3, ab % 3
    for it, t in enumerate(tiles):
        G = tile_global_indices(w, t)
        GA = G[pairs[:, 0]][:, None]
        GB = G[pairs[:, 1]][:, None]
        r = 3 * GA + a[None, :]
        c = 3 * GB + b[None, :]
        v = blocks[it]
        rows.append(r.ravel()); cols.append(c.ravel()); vals.append(v.ravel())
        off = pairs[:, 0] != pairs[:, 1]
        rows.append(c[off].ravel()); cols.append(r[off].ravel()); vals.append(v[off].ravel())
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def csr_from_coo(n: int, rows, cols, vals):
    """Sorted-unique pattern with values summed in the given order (np.add.at is sequential)."""
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    uniq, inv = np.unique(key, return_inverse=True)
    data = np.zeros(len(uniq))
    np.add.at(data, inv, vals)
    r = uniq // n
    c = uniq % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, c.astype(np.int32), data


def assemble_csr(w, pairs, blocks):
    """Global K (row_ptr int64, col_idx int32, values f64) from all tile blocks."""
    n = n_global_dofs(w)
    rows, cols, vals = coo_entries(w, pairs, blocks)
    return csr_from_coo(n, rows, cols, vals)


def csr_pattern(w, pairs):
    """Pattern only (row_ptr, col_idx), brute force over every tile."""
    dummy = np.zeros((w.n_tiles, len(pairs), 9))
    rp, ci, _ = assemble_csr(w, pairs, dummy)
    return rp, ci


def tiles_of_dof(w, G: int):
    """Tiles whose control net contains global control point G (ascending)."""
    from .geometry import global_grid, tile_shape
    GX, GY, GZ = global_grid(w)
    nx, ny, nz = tile_shape(w)
    g = (G % GX, (G // GX) % GY, G // (GX * GY))
    n = (nx, ny, nz)
    cand = []
    for k in range(3):
        m = n[k] - 1
        lst = [t for t in range(w.tiles[k]) if t * m <= g[k] <= t * m + m]
        cand.append(lst)
    Tx, Ty, _ = w.tiles
    return sorted(tx + Tx * (ty + Ty * tz) for tz in cand[2] for ty in cand[1] for tx in cand[0])


def csr_rows(w, pairs, block_of_tile, rows):
    """Sampled CSR rows computed one by one: for each requested row r, its sorted columns and
    values, summing the contributing tiles in ascending order.  block_of_tile(t) -> (n_nz, 9)."""
    out = {}
    for r in rows:
        G, a = divmod(int(r), 3)
        acc = {}
        for t in tiles_of_dof(w, G):
            Gt = tile_global_indices(w, t)
            A = int(np.nonzero(Gt == G)[0][0])
            blk = block_of_tile(t)
            for p, (P0, P1) in enumerate(pairs):
                if P0 == A:
                    for b in range(3):
                        c = 3 * int(Gt[P1]) + b
                        acc[c] = acc.get(c, 0.0) + blk[p, 3 * a + b]
                if P1 == A and P0 != A:
                    for b in range(3):
                        c = 3 * int(Gt[P0]) + b
                        acc[c] = acc.get(c, 0.0) + blk[p, 3 * b + a]
        cols = np.array(sorted(acc), dtype=np.int64)
        out[int(r)] = (cols, np.array([acc[c] for c in cols]))
    return out


def spmv(row_ptr, col_idx, vals, x):
    import scipy.sparse as sp
    n = len(row_ptr) - 1
    return sp.csr_matrix((vals, col_idx, row_ptr), shape=(n, n)) @ x


def to_scipy(row_ptr, col_idx, vals):
    import scipy.sparse as sp
    n = len(row_ptr) - 1
    return sp.csr_matrix((vals, col_idx.astype(np.int64), row_ptr), shape=(n, n))


def dense_global(w, pairs, blocks):
    """Dense global matrix by adding dense tile matrices (small cases only)."""
    n = n_global_dofs(w)
    nT = int(np.prod(w.tile.n_ctrl))
    K = np.zeros((n, n))
    for t in range(w.n_tiles):
        d = tile_dofs(w, t)
        K[np.ix_(d, d)] += tile_dense(pairs, blocks[t], nT)
    return K


def linop_apply(w, pairs: np.ndarray, blocks: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Matrix-free product of Section 4.2, eq. (74): K u = sum_t scatter(K^(t) u^(t)), with the
    tile matrices K^(t) built from the tile blocks (never the global matrix); tile products
    summed into the global vector in ascending tile order."""
    nT = int(np.prod(w.tile.n_ctrl))
    y = np.zeros(n_global_dofs(w))
    for t in range(len(blocks)):
        dofs = tile_dofs(w, t)
        yt = tile_dense(pairs, blocks[t], nT) @ u[dofs]
        np.add.at(y, dofs, yt)
    return y
