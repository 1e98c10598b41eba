"""Micro-scale stiffness lookup table (oracle, test infrastructure only).

Section 3.2.3:
  I_coo = {(A, B): A <= B, supp R_A and supp R_B share a micro element}   eq. (56)
  table[p(A,B), 9 C + 3 i + j] = int_{Omega_T} d_i(R_A o T^-1) d_j(R_B o T^-1) N_C dxi   eq. (52), (57)

The integral is pulled back to the tile parameter domain (xi = T^r(theta)):
  int_[0,1]^3 (J_T^-T grad_theta R_A)_i (J_T^-T grad_theta R_B)_j N_C(T^r(theta)) det J_T dtheta,
evaluated with n_g Gauss-Legendre points per direction on every micro element.
Tile-local indices are x-fastest, A = i + n_x (j + n_y k); pairs are sorted by (A, B).
"""
from __future__ import annotations

import itertools

import numpy as np

from .basis import bspline_basis, gauss01, nonempty_spans, support_elements
from .projection import bernstein3, n_pi


def micro_elements(tile):
    """List of micro elements as (x-span, y-span, z-span) index triples, x fastest, with their boxes."""
    spans = [nonempty_spans(tile.knots[k]) for k in range(3)]
    out = []
    for ez, ey, ex in itertools.product(range(len(spans[2])), range(len(spans[1])), range(len(spans[0]))):
        out.append(((ex, ey, ez), (spans[0][ex], spans[1][ey], spans[2][ez])))
    return out


def active_functions(tile, e):
    """Tile-local flat indices of the basis functions that are non-zero on micro element e (sorted)."""
    nx, ny, nz = tile.n_ctrl
    sup = [support_elements(tile.knots[k], tile.degree[k]) for k in range(3)]
    ax = [i for i in range(nx) if e[0] in sup[0][i]]
    ay = [j for j in range(ny) if e[1] in sup[1][j]]
    az = [k for k in range(nz) if e[2] in sup[2][k]]
    return sorted(i + nx * (j + ny * k) for k in az for j in ay for i in ax)


def pair_set(tile):
    """I_coo (eq. (56)) as an (n_nz, 2) int array, lexicographically sorted, by brute force over elements."""
    pairs = set()
    for e, _ in micro_elements(tile):
        act = active_functions(tile, e)
        for A in act:
            for B in act:
                if A <= B:
                    pairs.add((A, B))
    return np.array(sorted(pairs), dtype=np.int64)


def element_points(tile, box, n_g):
    """Gauss points of one micro element: basis values/gradients of all tile functions, map and Jacobian.

    Returns (R (G, n_T), dR (G, n_T, 3), X (G, 3), J (G, 3, 3), w (G,)) with J[c, k] = dT_c/dtheta_k.
    """
    xg, wg = gauss01(n_g)
    axes = []
    for k in range(3):
        lo, hi = box[k]
        pts = lo + (hi - lo) * xg
        N, dN = bspline_basis(tile.knots[k], tile.degree[k], pts, deriv=True)
        axes.append((N, dN, (hi - lo) * wg))
    (Nx, dNx, wx), (Ny, dNy, wy), (Nz, dNz, wz) = axes
    # point index g = gx + n_g (gy + n_g gz); function index A = i + nx (j + ny k)
    R = np.einsum("zk,yj,xi->zyxkji", Nz, Ny, Nx)
    Rx = np.einsum("zk,yj,xi->zyxkji", Nz, Ny, dNx)
    Ry = np.einsum("zk,yj,xi->zyxkji", Nz, dNy, Nx)
    Rz = np.einsum("zk,yj,xi->zyxkji", dNz, Ny, Nx)
    G = n_g ** 3
    R = R.reshape(G, -1)
    dR = np.stack([Rx.reshape(G, -1), Ry.reshape(G, -1), Rz.reshape(G, -1)], axis=-1)
    ctrl = tile.ctrl.reshape(-1, 3)
    X = R @ ctrl
    J = np.einsum("gAk,Ac->gck", dR, ctrl)
    w = np.einsum("z,y,x->zyx", wz, wy, wx).reshape(-1)
    return R, dR, X, J, w


def stiffness_table(tile, q, n_g: int, pairs=None) -> np.ndarray:
    """mat[K] of eq. (57): shape (n_nz, 9 n_pi), rows ordered as ``pairs``; q an int or a triple."""
    if pairs is None:
        pairs = pair_set(tile)
    nT = int(np.prod(tile.n_ctrl))
    pidx = -np.ones((nT, nT), dtype=np.int64)
    pidx[pairs[:, 0], pairs[:, 1]] = np.arange(len(pairs))
    npi = n_pi(q)
    table = np.zeros((len(pairs), 9 * npi))
    for e, box in micro_elements(tile):
        act = np.array(active_functions(tile, e))
        R, dR, X, J, w = element_points(tile, box, n_g)
        det = np.linalg.det(J)
        if np.any(det <= 0):
            raise ValueError("reference tile map is not positively oriented")
        # gradient w.r.t. xi = T^r(theta):  J^-T grad_theta R
        gxi = np.einsum("gkc,gAk->gAc", np.linalg.inv(J), dR[:, act, :])
        N = bernstein3(q, X)                                     # (G, n_pi)
        wd = w * det
        # full[a, i, C, b, j] = sum_g wd gxi[g,a,i] N[g,C] gxi[g,b,j]
        left = np.einsum("g,gai,gC->aiCg", wd, gxi, N).reshape(-1, len(wd))
        full = (left @ gxi.reshape(len(wd), -1)).reshape(len(act), 3, npi, len(act), 3)
        full = full.transpose(0, 3, 2, 1, 4).reshape(len(act), len(act), 9 * npi)  # [a, b, (C,i,j)]
        Aa, Bb = np.meshgrid(np.arange(len(act)), np.arange(len(act)), indexing="ij")
        sel = act[Aa] <= act[Bb]
        p = pidx[act[Aa][sel], act[Bb][sel]]
        if np.any(p < 0):
            raise AssertionError("pair missing from I_coo")
        table[p] += full[Aa[sel], Bb[sel]]
    return table
