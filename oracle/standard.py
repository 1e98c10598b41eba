"""Standard procedure: element loop with full Gauss quadrature (oracle, test infrastructure only).

This is the reference operator K^bullet of Section 3.3 (eq. (62)): on every tile,
every micro element and every Gauss point theta,
  xbar = T^r(theta),  J = J_M^(t)(xbar) J_T(theta),  grad_x R = J^-T grad_theta R,
  K_e += B^T D B det J w
with the engineering strain-displacement matrix B (rows xx, yy, zz, yz, xz, xy)
and the isotropic elasticity matrix D.  No macro field, no projection, no table:
the composition (eq. (10)) is evaluated pointwise.
"""
from __future__ import annotations

import numpy as np

from .geometry import eval_volume_points, tile_boxes, tile_index
from .macro_field import lame
from .tables import active_functions, element_points, micro_elements


def elasticity_matrix(lam, mu):
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def b_matrix(gx):
    """Strain-displacement matrix (6, 3 n) for gradients gx (n, 3), dof order (A, a) -> 3A + a."""
    n = gx.shape[0]
    B = np.zeros((6, 3 * n))
    B[0, 0::3] = gx[:, 0]
    B[1, 1::3] = gx[:, 1]
    B[2, 2::3] = gx[:, 2]
    B[3, 1::3] = gx[:, 2]; B[3, 2::3] = gx[:, 1]
    B[4, 0::3] = gx[:, 2]; B[4, 2::3] = gx[:, 0]
    B[5, 0::3] = gx[:, 1]; B[5, 1::3] = gx[:, 0]
    return B


def tile_matrix_standard(w, t: int, n_g: int = None) -> np.ndarray:
    """Dense (3 n_T, 3 n_T) stiffness of tile t by full Gauss quadrature of the composed geometry."""
    n_g = w.n_gauss if n_g is None else n_g
    lam, mu = lame(w.E, w.nu)
    D = elasticity_matrix(lam, mu)
    boxes = tile_boxes(w)
    tx, ty, tz = tile_index(w, t)
    a = np.array([boxes[0][0][tx], boxes[1][0][ty], boxes[2][0][tz]])
    h = np.array([boxes[0][1][tx], boxes[1][1][ty], boxes[2][1][tz]])
    nT = int(np.prod(w.tile.n_ctrl))
    K = np.zeros((3 * nT, 3 * nT))
    for e, box in micro_elements(w.tile):
        act = np.array(active_functions(w.tile, e))
        R, dR, X, JT, wts = element_points(w.tile, box, n_g)
        _, JM = eval_volume_points(w.macro.degree, w.macro.knots, w.macro.ctrl, a + h * X, weights=w.macro.weights)
        JM = JM * h[None, None, :]
        J = JM @ JT
        det = np.linalg.det(J)
        if np.any(det <= 0):
            raise ValueError(f"degenerate composed map in tile {t}")
        dofs = (3 * act[:, None] + np.arange(3)[None, :]).ravel()
        Ke = np.zeros((len(dofs), len(dofs)))
        Jinv = np.linalg.inv(J)
        for g in range(len(wts)):
            gx = dR[g, act, :] @ Jinv[g]       # row A: (J^-T grad R_A)^T
            B = b_matrix(gx)
            Ke += (B.T @ D @ B) * det[g] * wts[g]
        K[np.ix_(dofs, dofs)] += Ke
    return K


def tile_block_standard(w, t: int, pairs: np.ndarray, n_g: int = None) -> np.ndarray:
    """The same tile matrix in the upper-pair block layout (n_nz, 9)."""
    K = tile_matrix_standard(w, t, n_g)
    out = np.empty((len(pairs), 9))
    for p, (A, B) in enumerate(pairs):
        out[p] = K[3 * A:3 * A + 3, 3 * B:3 * B + 3].ravel()
    return out
