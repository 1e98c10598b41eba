"""Macro-scale L2 projection onto Bernstein polynomials (oracle, test infrastructure only).

Section 3.1.2, eq. (20)-(24) and eq. (42): the projection coefficients d of a
field f on [0,1]^3 solve  M_pi d = r  with  M_pi[k,l] = int N_k N_l  and
r_k = int N_k f,  N_C(xi) = B_c1(xi_1) B_c2(xi_2) B_c3(xi_3),
C = c1 + (q+1)(c2 + (q+1) c3).  Both integrals use the same n_fit-point
Gauss-Legendre rule per direction (n_fit >= q+1 keeps M_pi exact).  The 3-D
system is assembled and solved as a dense (q+1)^3 system -- no tensor
factorisation.

The fields projected are the 81 components of A_ij,ab (eq. (37)) on each tile,
which gives the right-hand operand of eq. (58):
  Coef^(t)[9 C + 3 i + j, 3 a + b] = <A_ij,ab^(t)>_C.
"""
from __future__ import annotations

import numpy as np

from .basis import bernstein, gauss01
from .geometry import eval_volume_grid, tile_boxes, tile_index
from .macro_field import lame, macro_field


def degrees(q):
    """Projection degrees per direction: an int q is (q, q, q); a triple is anisotropic (the
    paper's (3, 3, 4) for the twisted square)."""
    if np.ndim(q) == 0:
        return (int(q),) * 3
    return tuple(int(v) for v in q)


def n_pi(q) -> int:
    """Dimension of the projection space, prod_k (q_k + 1) (eq. (21))."""
    return int(np.prod([d + 1 for d in degrees(q)]))


def bernstein3(q, pts: np.ndarray) -> np.ndarray:
    """N_C at points pts (P, 3); column C = c1 + (q1+1)(c2 + (q2+1) c3), degrees q per direction."""
    qx, qy, qz = degrees(q)
    B1 = bernstein(qx, pts[:, 0])
    B2 = bernstein(qy, pts[:, 1])
    B3 = bernstein(qz, pts[:, 2])
    return np.einsum("pk,pj,pi->pkji", B3, B2, B1).reshape(len(pts), -1)


def fit_points(n_fit: int):
    """Tensor Gauss-Legendre points (x fastest) and weights on [0,1]^3."""
    x, wx = gauss01(n_fit)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    WZ, WY, WX = np.meshgrid(wx, wx, wx, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return pts, (WX * WY * WZ).ravel()


def projection_operator(q, n_fit: int) -> np.ndarray:
    """Matrix P (n_pi x n_fit^3) with d = P f(samples): P = M_pi^-1 N^T W (eq. (23)-(24))."""
    pts, wts = fit_points(n_fit)
    N = bernstein3(q, pts)                    # (S, n_pi)
    M = N.T @ (wts[:, None] * N)              # eq. (24) mass matrix
    return np.linalg.solve(M, N.T * wts[None, :])


def tile_macro_jacobians(w, t: int):
    """Jacobian of M^(t)(xi) = M(a + h xi) at the fit points of tile t, shape (S, 3, 3)."""
    boxes = tile_boxes(w)
    tx, ty, tz = tile_index(w, t)
    x, _ = gauss01(w.n_fit)
    a = [boxes[0][0][tx], boxes[1][0][ty], boxes[2][0][tz]]
    h = [boxes[0][1][tx], boxes[1][1][ty], boxes[2][1][tz]]
    _, J = eval_volume_grid(w.macro.degree, w.macro.knots, w.macro.ctrl,
                            a[0] + h[0] * x, a[1] + h[1] * x, a[2] + h[2] * x, weights=w.macro.weights)
    J = J.reshape(-1, 3, 3) * np.array(h)[None, None, :]
    return J


def tile_coefficients(w, t: int, P=None) -> np.ndarray:
    """Coef^(t), shape (9 n_pi, 9): rows 9C+3i+j, columns 3a+b."""
    lam, mu = lame(w.E, w.nu)
    if P is None:
        P = projection_operator(w.q, w.n_fit)
    J = tile_macro_jacobians(w, t)
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError(f"degenerate macro element at tile {t}")
    A = macro_field(J, lam, mu).reshape(len(J), 81)   # [s, (i,j,a,b)]
    d = P @ A                                          # [C, (i,j,a,b)]
    d = d.reshape(-1, 3, 3, 3, 3)                      # [C, i, j, a, b]
    return d.reshape(-1, 9)                            # rows (C, i, j), cols (a, b)


def all_coefficients(w, tiles=None) -> np.ndarray:
    """Stack of Coef^(t) for the listed tiles (default all), shape (T, 9 n_pi, 9)."""
    P = projection_operator(w.q, w.n_fit)
    tiles = range(w.n_tiles) if tiles is None else tiles
    return np.stack([tile_coefficients(w, int(t), P) for t in tiles])
