"""Projection error of the macro field and the adaptive choice of the projection degree
(oracle, test infrastructure only).

Section 3.3.1, eq. (59): E_proj = max over tiles and over the tile's box of
|A(xi) - Pi A(xi)|_F / |A(xi)|_F, A the macro field of eq. (37) and Pi A its projection onto the
Bernstein space Q_q (the fitted coefficients of eq. (42), the same as the stiffness assembly's).
Section 3.2.2 (after eq. (48)) evaluates the error by sampling; here the maximum runs over a
uniform tensor grid of n_s points per direction with both ends, x_k = k / (n_s - 1), in every
tile's box coordinates.  Eq. (65): the degree is the first q, counting up from the macro map's
degree, with E_proj(q) <= tol; the fit uses q + 1 Gauss-Legendre points per direction.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .geometry import eval_volume_grid, tile_boxes, tile_index
from .macro_field import lame, macro_field
from .projection import bernstein3, degrees, tile_coefficients


def sample_grid(n_s: int) -> np.ndarray:
    """Uniform points with both ends, 1-D."""
    return np.linspace(0.0, 1.0, n_s)


def tile_field_at(w, t: int, x1: np.ndarray) -> np.ndarray:
    """Exact A at the tensor grid x1^3 of tile t's box coordinates (x fastest), shape (S, 81)."""
    lam, mu = lame(w.E, w.nu)
    boxes = tile_boxes(w)
    tx, ty, tz = tile_index(w, t)
    a = [boxes[0][0][tx], boxes[1][0][ty], boxes[2][0][tz]]
    h = [boxes[0][1][tx], boxes[1][1][ty], boxes[2][1][tz]]
    _, J = eval_volume_grid(w.macro.degree, w.macro.knots, w.macro.ctrl,
                            a[0] + h[0] * x1, a[1] + h[1] * x1, a[2] + h[2] * x1, weights=w.macro.weights)
    J = J.reshape(-1, 3, 3) * np.array(h)[None, None, :]
    return macro_field(J, lam, mu).reshape(len(J), 81)


def tile_eproj(w, t: int, n_s: int) -> float:
    """max over the samples of tile t of |A - Pi A|_F / |A|_F (eq. (59))."""
    x1 = sample_grid(n_s)
    A = tile_field_at(w, t, x1)                                   # (S, 81), (i, j, a, b)
    coef = tile_coefficients(w, t)                                # rows 9C+3i+j, cols 3a+b
    Z, Y, X = np.meshgrid(x1, x1, x1, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    B = bernstein3(w.q, pts)                                      # (S, n_pi)
    PA = np.einsum("sC,Cijab->sijab", B, coef.reshape(-1, 3, 3, 3, 3)).reshape(len(pts), 81)
    return float(np.max(np.linalg.norm(A - PA, axis=1) / np.linalg.norm(A, axis=1)))


def eproj(w, q=None, n_s: int = 5) -> float:
    """E_proj (eq. (59)) at projection degree q (default w.q; an int or a triple), fit on
    max_k q_k + 1 points per direction (a least-squares fit in the directions of lower degree)."""
    if q is not None:
        w = dataclasses.replace(w, q=q, n_fit=max(degrees(q)) + 1)
    return max(tile_eproj(w, t, n_s) for t in range(w.n_tiles))


def select_q(w, tol: float, q_max: int = 6, n_s: int = 5):
    """Eq. (65): the first q >= the macro degree with E_proj(q) <= tol; (q, E_proj(q)), or
    (None, E_proj(q_max)) if no degree up to q_max meets tol."""
    q0 = max(w.macro.degree)
    e = None
    for q in range(q0, q_max + 1):
        e = eproj(w, q, n_s)
        if e <= tol:
            return q, e
    return None, e


def select_q_aniso(w, tol: float, q_max: int = 6, n_s: int = 5):
    """The anisotropic reading of eq. (65) (the paper's twisted square, degrees (3, 3, 4)): start
    from the macro map's degrees per direction; while E_proj > tol, raise by one the direction
    whose raise gives the lowest E_proj (ties: the lowest direction index), up to q_max each.
    Returns (degrees, E_proj) or (None, E_proj of the last degrees tried)."""
    q = list(w.macro.degree)
    e = eproj(w, tuple(q), n_s)
    while e > tol:
        best = None
        for k in range(3):
            if q[k] >= q_max:
                continue
            trial = list(q)
            trial[k] += 1
            et = eproj(w, tuple(trial), n_s)
            if best is None or et < best[0]:
                best = (et, trial)
        if best is None:
            return None, e
        e, q = best
    return tuple(q), e
