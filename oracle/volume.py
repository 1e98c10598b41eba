"""Volume of the microstructured geometry and its shape sensitivity (oracle, test infrastructure only).

Section 3.1, the illustrative example of the method:
* eq. (14): V^(t) = int over the tile parameter domain of |det J_T| |det J_M^(t) o T| dtheta;
* eq. (15), (23)-(24): |det J_M^(t)| projected onto the Bernstein space Q_q, coefficients d^(t);
* eq. (18): the table t^h[C] = int |det J_T| (N_C o T) dtheta (micro elements, Gauss points);
* eq. (17), (19): V^(t) ~ t^h . d^(t), V = sum_t V^(t) (tiles in ascending order);
* eq. (25)-(26): the folded table t_pi = M_pi^-1 t^h, with V^(t) = t_pi . r^(t),
  r^(t)[k] = int N_k |det J_M^(t)| dxi (the right-hand side of eq. (24)).
Section 4.1.1, eq. (66)-(67): dV^(t)/dm = int v(xi) d|det J_M^(t)|/dm (xi) dxi with the adjoint
field v = sum_C N_C t_pi[C]; the integral uses the same Gauss rule (n_fit points per direction) as
r^(t), so it is the exact derivative of the discrete V.  With J = J_M(a + h xi) diag(h) and
J[c][n] = sum_i m_(i,c) h_n d_n N_i: d det J / d m_(i,c) = det J sum_n (J^-1)[n][c] h_n d_n N_i.
Maps are orientation-preserving (det J > 0), as in the rest of the oracle.
"""
from __future__ import annotations

import numpy as np

from .basis import bspline_basis, gauss01
from .geometry import control_point_gradient, tile_boxes, tile_index
from .projection import bernstein3, degrees, fit_points, n_pi, projection_operator, tile_macro_jacobians
from .tables import element_points, micro_elements


def volume_table(tile, q, n_g: int) -> np.ndarray:
    """t^h (eq. (18)), shape (n_pi,); q an int or a degree triple."""
    t = np.zeros(n_pi(q))
    for _, box in micro_elements(tile):
        _, _, X, JT, wts = element_points(tile, box, n_g)
        t += (wts * np.abs(np.linalg.det(JT))) @ bernstein3(q, X)
    return t


def mass_matrix(q) -> np.ndarray:
    """M_pi (eq. (24)): int N_k N_l over [0,1]^3 by a Gauss rule exact for degree 2 max q."""
    pts, wts = fit_points(max(degrees(q)) + 1)
    N = bernstein3(q, pts)
    return N.T @ (wts[:, None] * N)


def folded_table(q, t_h: np.ndarray) -> np.ndarray:
    """t_pi = M_pi^-1 t^h (eq. (26))."""
    return np.linalg.solve(mass_matrix(q), t_h)


def tile_detJ(w, t: int) -> np.ndarray:
    """|det J_M^(t)| at the fit points (x fastest)."""
    return np.abs(np.linalg.det(tile_macro_jacobians(w, t)))


def tile_volumes(w, t_h: np.ndarray) -> np.ndarray:
    """V^(t) = t^h . d^(t) (eq. (17)), d^(t) the projection of |det J_M^(t)| (eq. (15), (23))."""
    P = projection_operator(w.q, w.n_fit)
    return np.array([t_h @ (P @ tile_detJ(w, t)) for t in range(w.n_tiles)])


def volume(w, t_h: np.ndarray) -> float:
    """V (eq. (19)): the tile volumes summed in ascending tile order."""
    v = 0.0
    for x in tile_volumes(w, t_h):
        v += x
    return v


def volume_folded(w, t_pi: np.ndarray) -> float:
    """V = sum_t t_pi . r^(t) (eq. (25)), r^(t) by the n_fit-point Gauss rule."""
    pts, wts = fit_points(w.n_fit)
    N = bernstein3(w.q, pts)
    return float(sum(t_pi @ (N.T @ (wts * tile_detJ(w, t))) for t in range(w.n_tiles)))


def volume_standard(w, n_g: int = None) -> float:
    """V by eq. (14) directly: Gauss quadrature over the micro elements of every tile."""
    n_g = w.n_gauss if n_g is None else n_g
    from .geometry import eval_volume_points
    boxes = tile_boxes(w)
    v = 0.0
    for t in range(w.n_tiles):
        tx, ty, tz = tile_index(w, t)
        a = np.array([boxes[0][0][tx], boxes[1][0][ty], boxes[2][0][tz]])
        h = np.array([boxes[0][1][tx], boxes[1][1][ty], boxes[2][1][tz]])
        for _, box in micro_elements(w.tile):
            _, _, X, JT, wts = element_points(w.tile, box, n_g)
            _, JM = eval_volume_points(w.macro.degree, w.macro.knots, w.macro.ctrl, a + h * X, weights=w.macro.weights)
            v += float(np.sum(wts * np.abs(np.linalg.det(JT)) * np.abs(np.linalg.det(JM * h[None, None, :]))))
    return v


def adjoint_field(q, t_pi: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """v(xi) = sum_C N_C(xi) t_pi[C] (eq. (67)) at points pts (P, 3)."""
    return bernstein3(q, pts) @ t_pi


def volume_grad(w, t_pi: np.ndarray) -> np.ndarray:
    """dV/dm (eq. (66)), shape (n_z, n_y, n_x, 3) like the macro control points; for a NURBS map
    the derivative of J by a control point is the rational basis' gradient (weights fixed)."""
    nz, ny, nx = w.macro.ctrl.shape[:3]
    grad = np.zeros((nz, ny, nx, 3))
    xg, _ = gauss01(w.n_fit)
    pts, wts = fit_points(w.n_fit)
    v = adjoint_field(w.q, t_pi, pts)
    boxes = tile_boxes(w)
    nf = w.n_fit
    for t in range(w.n_tiles):
        tx, ty, tz = tile_index(w, t)
        a = [boxes[0][0][tx], boxes[1][0][ty], boxes[2][0][tz]]
        h = [boxes[0][1][tx], boxes[1][1][ty], boxes[2][1][tz]]
        J = tile_macro_jacobians(w, t)                   # (S, 3, 3), includes diag(h)
        D = np.linalg.det(J)
        F = np.linalg.inv(J)
        # per sample s = sx + nf (sy + nf sz): G[s, c, n] = w_s v_s D_s F[n, c] h_n
        G = (wts * v * D)[:, None, None] * np.transpose(F, (0, 2, 1)) * np.array(h)[None, None, :]
        G = G.reshape(nf, nf, nf, 3, 3)                  # (sz, sy, sx, c, n)
        grad += control_point_gradient(w.macro.knots, w.macro.degree, w.macro.weights,
                                       a[0] + h[0] * xg, a[1] + h[1] * xg, a[2] + h[2] * xg, G)
    return grad
