"""Spline volumes, tile boxes and global numbering (oracle, test infrastructure only).

* Trivariate B-spline map S(x) = sum_i R_i(x) s_i (eq. (2)); the reference tile
  T^r (eq. (3)) and the macro map M (eq. (4)) are both of this form.
* Macro sub-domains (eq. (5)-(8)): tile t occupies the parameter box
  B_t = prod_k [a_k, a_k + h_k]; its macro element map is M^(t)(xi) = M(a + h*xi),
  which is the Bezier element of eq. (7)-(8) when the box is a knot span.
* Conforming C0 gluing of tiles: tile-local control point (i, j, k) of tile
  (tx, ty, tz) has global index (tx (n_x-1) + i, ty (n_y-1) + j, tz (n_z-1) + k),
  x fastest; degree of freedom 3 G + a.
"""
from __future__ import annotations

import numpy as np

from .basis import bspline_basis, n_basis, nonempty_spans


def _rational(X, J, W, dW):
    """Quotient rule for a NURBS map from the homogeneous sums A = sum w N P (X, J here) and
    W = sum w N: M = A / W, dM/dx_k = (dA/dx_k - M dW/dx_k) / W."""
    M = X / W[..., None]
    Jr = (J - M[..., :, None] * dW[..., None, :]) / W[..., None, None]
    return M, Jr


def rational_grid_terms(knots, degree, weights, xs, ys, zs):
    """Basis tensors of a NURBS control-point derivative on the grid xs x ys x zs: the 1-D
    B-spline values and derivatives per direction, and W = sum w N with its gradient
    (shapes (len(zs), len(ys), len(xs)) and (..., 3)).  With R_i = w_i N_i / W,
    d_n R_i = w_i (d_n N_i - N_i d_n W / W) / W."""
    Bx, dBx = bspline_basis(knots[0], degree[0], xs, deriv=True)
    By, dBy = bspline_basis(knots[1], degree[1], ys, deriv=True)
    Bz, dBz = bspline_basis(knots[2], degree[2], zs, deriv=True)
    wt = np.asarray(weights, dtype=np.float64)
    W = np.einsum("zk,yj,xi,kji->zyx", Bz, By, Bx, wt, optimize=True)
    dW = np.stack([np.einsum("zk,yj,xi,kji->zyx", Bz, By, dBx, wt, optimize=True),
                   np.einsum("zk,yj,xi,kji->zyx", Bz, dBy, Bx, wt, optimize=True),
                   np.einsum("zk,yj,xi,kji->zyx", dBz, By, Bx, wt, optimize=True)], axis=-1)
    return (Bx, dBx), (By, dBy), (Bz, dBz), W, dW


def control_point_gradient(knots, degree, weights, xs, ys, zs, G):
    """g[k, j, i, c] = sum over the grid s of sum_n G[s, c, n] d_n R_(i,j,k)(s), G of shape
    (len(zs), len(ys), len(xs), 3, 3) (n: the parameter direction); R the B-spline basis when
    weights is None, else the NURBS basis."""
    if weights is None:
        Bx, dBx = bspline_basis(knots[0], degree[0], xs, deriv=True)
        By, dBy = bspline_basis(knots[1], degree[1], ys, deriv=True)
        Bz, dBz = bspline_basis(knots[2], degree[2], zs, deriv=True)
        g = np.einsum("zyxc,zk,yj,xi->kjic", G[..., 0], Bz, By, dBx)
        g += np.einsum("zyxc,zk,yj,xi->kjic", G[..., 1], Bz, dBy, Bx)
        g += np.einsum("zyxc,zk,yj,xi->kjic", G[..., 2], dBz, By, Bx)
        return g
    (Bx, dBx), (By, dBy), (Bz, dBz), W, dW = rational_grid_terms(knots, degree, weights, xs, ys, zs)
    Gw = G / W[..., None, None]
    H = np.einsum("zyxcn,zyxn->zyxc", G, dW) / (W * W)[..., None]
    g = np.einsum("zyxc,zk,yj,xi->kjic", Gw[..., 0], Bz, By, dBx)
    g += np.einsum("zyxc,zk,yj,xi->kjic", Gw[..., 1], Bz, dBy, Bx)
    g += np.einsum("zyxc,zk,yj,xi->kjic", Gw[..., 2], dBz, By, Bx)
    g -= np.einsum("zyxc,zk,yj,xi->kjic", H, Bz, By, Bx)
    return g * np.asarray(weights, dtype=np.float64)[..., None]


def eval_volume_grid(degree, knots, ctrl, xs, ys, zs, weights=None):
    """Map value X and Jacobian J on the tensor grid xs x ys x zs (each 1-D).

    ctrl has shape (n_z, n_y, n_x, 3); weights (n_z, n_y, n_x) makes the map a NURBS
    (R_i = w_i N_i / sum_j w_j N_j).  Returns X with shape (len(zs), len(ys), len(xs), 3)
    and J with shape (len(zs), len(ys), len(xs), 3, 3), J[..., c, k] = d X_c / d x_k.
    """
    Bx, dBx = bspline_basis(knots[0], degree[0], xs, deriv=True)
    By, dBy = bspline_basis(knots[1], degree[1], ys, deriv=True)
    Bz, dBz = bspline_basis(knots[2], degree[2], zs, deriv=True)
    c = np.asarray(ctrl, dtype=np.float64)
    if weights is not None:
        wt = np.asarray(weights, dtype=np.float64)
        c = c * wt[..., None]
    X = np.einsum("zk,yj,xi,kjic->zyxc", Bz, By, Bx, c, optimize=True)
    J = np.empty(X.shape + (3,))
    J[..., 0] = np.einsum("zk,yj,xi,kjic->zyxc", Bz, By, dBx, c, optimize=True)
    J[..., 1] = np.einsum("zk,yj,xi,kjic->zyxc", Bz, dBy, Bx, c, optimize=True)
    J[..., 2] = np.einsum("zk,yj,xi,kjic->zyxc", dBz, By, Bx, c, optimize=True)
    if weights is None:
        return X, J
    W = np.einsum("zk,yj,xi,kji->zyx", Bz, By, Bx, wt, optimize=True)
    dW = np.stack([np.einsum("zk,yj,xi,kji->zyx", Bz, By, dBx, wt, optimize=True),
                   np.einsum("zk,yj,xi,kji->zyx", Bz, dBy, Bx, wt, optimize=True),
                   np.einsum("zk,yj,xi,kji->zyx", dBz, By, Bx, wt, optimize=True)], axis=-1)
    return _rational(X, J, W, dW)


def eval_volume_points(degree, knots, ctrl, pts, weights=None):
    """Map value and Jacobian at scattered points pts (P, 3) (weights as in eval_volume_grid)."""
    pts = np.asarray(pts, dtype=np.float64)
    Bx, dBx = bspline_basis(knots[0], degree[0], pts[:, 0], deriv=True)
    By, dBy = bspline_basis(knots[1], degree[1], pts[:, 1], deriv=True)
    Bz, dBz = bspline_basis(knots[2], degree[2], pts[:, 2], deriv=True)
    c = np.asarray(ctrl, dtype=np.float64)
    if weights is not None:
        wt = np.asarray(weights, dtype=np.float64)
        c = c * wt[..., None]
    X = np.einsum("pk,pj,pi,kjic->pc", Bz, By, Bx, c, optimize=True)
    J = np.empty(X.shape + (3,))
    J[..., 0] = np.einsum("pk,pj,pi,kjic->pc", Bz, By, dBx, c, optimize=True)
    J[..., 1] = np.einsum("pk,pj,pi,kjic->pc", Bz, dBy, Bx, c, optimize=True)
    J[..., 2] = np.einsum("pk,pj,pi,kjic->pc", dBz, By, Bx, c, optimize=True)
    if weights is None:
        return X, J
    W = np.einsum("pk,pj,pi,kji->p", Bz, By, Bx, wt, optimize=True)
    dW = np.stack([np.einsum("pk,pj,pi,kji->p", Bz, By, dBx, wt, optimize=True),
                   np.einsum("pk,pj,pi,kji->p", Bz, dBy, Bx, wt, optimize=True),
                   np.einsum("pk,pj,pi,kji->p", dBz, By, Bx, wt, optimize=True)], axis=-1)
    return _rational(X, J, W, dW)


def tile_boxes_1d(knots, n_tiles: int, box_mode: int):
    """Per-direction box origins a and sizes h for the tile grid.

    box_mode 0: tile i is the i-th non-empty knot span of the macro map (eq. (5)-(8));
    box_mode 1: uniform boxes of size 1/n_tiles.
    """
    if box_mode == 0:
        spans = nonempty_spans(knots)
        if len(spans) != n_tiles:
            raise ValueError("box_mode 0 needs one tile per non-empty macro knot span")
        a = np.array([s[0] for s in spans])
        h = np.array([s[1] - s[0] for s in spans])
        return a, h
    if box_mode == 1:
        a = np.arange(n_tiles) / n_tiles
        h = np.full(n_tiles, 1.0 / n_tiles)
        return a, h
    raise ValueError("unknown box mode")


def tile_boxes(w):
    """(a, h) arrays per direction for workload w."""
    return [tile_boxes_1d(w.macro.knots[k], w.tiles[k], w.box_mode) for k in range(3)]


def tile_index(w, t: int):
    Tx, Ty, _ = w.tiles
    return t % Tx, (t // Tx) % Ty, t // (Tx * Ty)


def tile_shape(w):
    """Tile control-net size per direction (n_x, n_y, n_z)."""
    return w.tile.n_ctrl


def global_grid(w):
    nx, ny, nz = tile_shape(w)
    Tx, Ty, Tz = w.tiles
    return (Tx * (nx - 1) + 1, Ty * (ny - 1) + 1, Tz * (nz - 1) + 1)


def n_global_dofs(w) -> int:
    g = global_grid(w)
    return 3 * g[0] * g[1] * g[2]


def tile_global_indices(w, t: int) -> np.ndarray:
    """Global control-point index G of every tile-local control point A (A x-fastest)."""
    nx, ny, nz = tile_shape(w)
    GX, GY, _ = global_grid(w)
    tx, ty, tz = tile_index(w, t)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    gx = tx * (nx - 1) + i
    gy = ty * (ny - 1) + j
    gz = tz * (nz - 1) + k
    return (gx + GX * (gy + GY * gz)).reshape(-1)


def tile_dofs(w, t: int) -> np.ndarray:
    """Global dof numbers of the tile-local dofs, ordered (A, a) -> 3 A + a."""
    G = tile_global_indices(w, t)
    return (3 * G[:, None] + np.arange(3)[None, :]).reshape(-1)


def composed_control_points(w) -> np.ndarray:
    """Physical position of every global control point: M(a_t + h_t * t_i) (used for rigid modes)."""
    nx, ny, nz = tile_shape(w)
    boxes = tile_boxes(w)
    GX, GY, GZ = global_grid(w)
    out = np.zeros((GX * GY * GZ, 3))
    tc = w.tile.ctrl.reshape(-1, 3)
    for t in range(w.n_tiles):
        tx, ty, tz = tile_index(w, t)
        a = np.array([boxes[0][0][tx], boxes[1][0][ty], boxes[2][0][tz]])
        h = np.array([boxes[0][1][tx], boxes[1][1][ty], boxes[2][1][tz]])
        X, _ = eval_volume_points(w.macro.degree, w.macro.knots, w.macro.ctrl, a + h * tc, w.macro.weights)
        out[tile_global_indices(w, t)] = X
    return out
