"""Shape sensitivity of u^T K^pi u with respect to the macro control points
(oracle, test infrastructure only).

Section 4.1.2, eq. (69)-(73): for the compliance c = f^T K^-1 f with a load that
does not move, dc/dm = -u^T (dK^pi/dm) u with u = K^-1 f.  The internal-work
derivative is the adjoint field (eq. (71)-(73)) -- the lookup table contracted
with products of displacement derivatives -- paired with dA/dm.

Chain used here, per tile t, written separately from any GPU code:
  u^T K^(t) u = sum_{C,i,j,a,b} Coef[(C,i,j),(a,b)] W[(C,i,j),(a,b)],
  W = table^T U,  U[p,(a,b)] = m_p u_(A,a) u_(B,b),  m_p = 2 if A < B else 1     (eq. (73))
  Coef = P A(samples)  (projection, eq. (23)-(24))  =>  dA(sample s) = P^T W
  dA/dJ by complex-step differentiation of the paper's curvilinear route (eq. (37)),
  J = J_M(a + h xi) diag(h)  =>  dJ/dm_k,c = e_c (grad N_k * h)^T.
The complex step makes dA/dJ exact to rounding without any hand-derived formula.
"""
from __future__ import annotations

import numpy as np

from .basis import bspline_basis, gauss01
from .geometry import control_point_gradient, tile_boxes, tile_dofs, tile_index
from .macro_field import lame, macro_field
from .projection import projection_operator, tile_coefficients, tile_macro_jacobians


def tile_U(pairs, ut):
    """U[p, 3a+b] = m_p u_(A,a) u_(B,b) for the tile displacement ut (n_T, 3)."""
    A, B = pairs[:, 0], pairs[:, 1]
    m = np.where(A < B, 2.0, 1.0)
    return m[:, None] * np.einsum("pa,pb->pab", ut[A], ut[B]).reshape(len(pairs), 9)


def uKu(w, table, pairs, u, tiles=None):
    """u^T K^pi u as the sum of per-tile terms (only the listed tiles, default all)."""
    P = projection_operator(w.q, w.n_fit)
    tiles = range(w.n_tiles) if tiles is None else tiles
    total = 0.0
    for t in tiles:
        ut = u[tile_dofs(w, t)].reshape(-1, 3)
        blk = table @ tile_coefficients(w, t, P)
        total += float(np.sum(blk * tile_U(pairs, ut)))
    return total


def _dA_dJ(J, lam, mu, h=1e-30):
    """Complex-step derivatives dA/dJ_mn, shape (S, 3, 3, 81): [s, m, n, comp]."""
    S = len(J)
    out = np.empty((S, 3, 3, 81))
    for m in range(3):
        for n in range(3):
            Jc = J.astype(np.complex128)
            Jc[:, m, n] += 1j * h
            out[:, m, n, :] = macro_field(Jc, lam, mu, signed_det=True).reshape(S, 81).imag / h
    return out


def tile_box(w, t):
    boxes = tile_boxes(w)
    tx, ty, tz = tile_index(w, t)
    a = np.array([boxes[0][0][tx], boxes[1][0][ty], boxes[2][0][tz]])
    h = np.array([boxes[0][1][tx], boxes[1][1][ty], boxes[2][1][tz]])
    return a, h


def grad_uKu(w, table, pairs, u, tiles=None):
    """d(u^T K^pi u)/d m, shape like w.macro.ctrl (n_z, n_y, n_x, 3) (NURBS: weights fixed)."""
    lam, mu = lame(w.E, w.nu)
    P = projection_operator(w.q, w.n_fit)
    x, _ = gauss01(w.n_fit)
    g = np.zeros_like(w.macro.ctrl)
    tiles = range(w.n_tiles) if tiles is None else tiles
    for t in tiles:
        ut = u[tile_dofs(w, t)].reshape(-1, 3)
        W = table.T @ tile_U(pairs, ut)                 # (9 n_pi, 9): rows (C,i,j), cols (a,b)
        Wc = W.reshape(-1, 3, 3, 3, 3).reshape(-1, 81)  # [C, (i,j,a,b)]
        Abar = P.T @ Wc                                 # [s, (i,j,a,b)]
        J = tile_macro_jacobians(w, t)
        dA = _dA_dJ(J, lam, mu)
        Jbar = np.einsum("sc,smnc->smn", Abar, dA)     # dL/dJ at each sample
        a, h = tile_box(w, t)
        pts = [a[k] + h[k] * x for k in range(3)]
        # J[s, c, n] = h_n sum_k m_k,c dR_k/dx_n ;  samples s = (sz, sy, sx), x fastest
        Jb = Jbar.reshape(len(x), len(x), len(x), 3, 3) * h[None, None, None, None, :]
        g += control_point_gradient(w.macro.knots, w.macro.degree, getattr(w.macro, "weights", None),
                                    pts[0], pts[1], pts[2], Jb)
    return g


def tiles_touching(w, k_index):
    """Tiles whose macro box meets the support of macro control point (i, j, k)."""
    from .basis import n_basis
    boxes = tile_boxes(w)
    out_axes = []
    for d in range(3):
        kn = w.macro.knots[d]
        p = w.macro.degree[d]
        i = k_index[d]
        lo, hi = kn[i], kn[i + p + 1]
        a, h = boxes[d]
        out_axes.append([tt for tt in range(len(a)) if a[tt] < hi and a[tt] + h[tt] > lo])
    Tx, Ty, _ = w.tiles
    return sorted(tx + Tx * (ty + Ty * tz) for tz in out_axes[2] for ty in out_axes[1] for tx in out_axes[0])
