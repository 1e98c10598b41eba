"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the benchmark.

This module builds *input data only*: knot vectors, control nets, tile grids,
material constants and the random draws that perturb them.  It contains none of
the assembly method's arithmetic (no basis evaluation, no Jacobians, no
quadrature), so both the CPU oracle and the HIP path can consume it without
sharing any of the method's code.

The paper's own geometries (its reference tiles, the quarter torus with a
three-circle section and the twisted square, Sections 3.3.2-3.3.4) are not
available, so every workload below is a stand-in with the shapes and sizes of
those experiments: a B-spline macro map (eq. (4)) on a tensor-product knot
grid, a single-patch B-spline reference tile (eq. (3)) whose boundary control
points sit at the identity position (so neighbouring tiles conform), and a tile
grid (Section 2.2.2).

Random draws follow one fixed order: macro-map jitter first, then tile
perturbations, both in x-fastest control-point order.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = [
    "Spline3D", "Workload", "open_knots", "greville", "make", "CONFIGS", "nurbs_quarter_torus", "nurbs_twisted_square",
    "tile_family", "family_params", "random_displacement",
]


@dataclass
class Spline3D:
    """A trivariate B-spline in plain arrays.

    degree[k], knots[k] (clamped, non-decreasing, on [0, 1]) for k = x, y, z and
    ctrl of shape (n_z, n_y, n_x, 3): control point (i, j, k) is ctrl[k, j, i].
    weights: None for a B-spline, else positive NURBS weights of shape (n_z, n_y, n_x).
    """
    degree: Tuple[int, int, int]
    knots: Tuple[np.ndarray, np.ndarray, np.ndarray]
    ctrl: np.ndarray
    weights: Optional[np.ndarray] = None

    @property
    def n_ctrl(self) -> Tuple[int, int, int]:
        return (self.ctrl.shape[2], self.ctrl.shape[1], self.ctrl.shape[0])

    def copy(self) -> "Spline3D":
        return Spline3D(tuple(self.degree), tuple(k.copy() for k in self.knots), self.ctrl.copy(),
                        None if self.weights is None else self.weights.copy())


@dataclass
class Workload:
    name: str
    macro: Spline3D
    tile: Spline3D
    tiles: Tuple[int, int, int]
    box_mode: int          # 0: tiles are the macro knot spans; 1: uniform parameter boxes
    q: int                 # projection degree p_pi
    n_fit: int             # fit samples per direction (Gauss-Legendre nodes)
    n_gauss: int           # Gauss-Legendre points per direction per micro element
    E: float = 1.0
    nu: float = 0.3
    seed: int = 0
    extra: Dict = field(default_factory=dict)

    @property
    def n_tiles(self) -> int:
        return int(np.prod(self.tiles))

    def with_tile(self, tile: Spline3D) -> "Workload":
        return replace(self, tile=tile)


def open_knots(degree: int, n_el: int) -> np.ndarray:
    """Uniform clamped knot vector on [0, 1] with n_el elements."""
    inner = [i / n_el for i in range(1, n_el)]
    return np.array([0.0] * (degree + 1) + inner + [1.0] * (degree + 1), dtype=np.float64)


def greville(knots: np.ndarray, degree: int) -> np.ndarray:
    """Greville abscissae: averages of `degree` consecutive interior knots."""
    n = len(knots) - degree - 1
    if degree == 0:
        return 0.5 * (knots[:-1] + knots[1:])[:n]
    return np.array([knots[i + 1:i + 1 + degree].mean() for i in range(n)], dtype=np.float64)


def _grid_points(gx: np.ndarray, gy: np.ndarray, gz: np.ndarray) -> np.ndarray:
    """(nz, ny, nx, 3) array of parameter triples, x fastest."""
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def _interior_mask(shape_zyx: Tuple[int, int, int]) -> np.ndarray:
    nz, ny, nx = shape_zyx
    m = np.zeros(shape_zyx, dtype=bool)
    m[1:nz - 1, 1:ny - 1, 1:nx - 1] = True
    return m


def identity_spline(degree: Tuple[int, int, int], n_el: Tuple[int, int, int]) -> Spline3D:
    """B-spline volume on [0,1]^3 whose control points are the Greville abscissae (the identity map)."""
    knots = tuple(open_knots(degree[k], n_el[k]) for k in range(3))
    g = [greville(knots[k], degree[k]) for k in range(3)]
    return Spline3D(tuple(degree), knots, _grid_points(*g))


def _jitter_interior(sp: Spline3D, rng: np.random.Generator, amp: float) -> None:
    mask = _interior_mask(sp.ctrl.shape[:3])
    n = int(mask.sum())
    sp.ctrl[mask] += rng.uniform(-amp, amp, size=(n, 3))


def _pull_interior(sp: Spline3D, rng: np.random.Generator, smax: float) -> None:
    """Pull every interior tile control point toward the tile centre: t <- t + s (c - t), s ~ U(0, smax)."""
    mask = _interior_mask(sp.ctrl.shape[:3])
    n = int(mask.sum())
    s = rng.uniform(0.0, smax, size=n)
    c = np.array([0.5, 0.5, 0.5])
    pts = sp.ctrl[mask]
    sp.ctrl[mask] = pts + s[:, None] * (c - pts)


def _mapped_spline(degree, n_el, fmap) -> Spline3D:
    """Control points placed at the image of the Greville abscissae under a closed-form map."""
    sp = identity_spline(degree, n_el)
    u, v, w = sp.ctrl[..., 0], sp.ctrl[..., 1], sp.ctrl[..., 2]
    sp.ctrl = np.stack(fmap(u, v, w), axis=-1)
    return sp


def _cantilever(u, v, w):
    # 10 x 2 x 2 box bent by a quarter arc; centre-line radius 20/pi keeps its length at 10.
    # The radius decreases with v so that the map is positively oriented.
    rc = 20.0 / np.pi
    phi = 0.5 * np.pi * u
    r = rc + (1.0 - 2.0 * v)
    return r * np.cos(phi), r * np.sin(phi), 2.0 * w


def _torus_sector(u, v, w):
    # quarter of a torus with a square 0.5 x 0.5 section around the unit circle,
    # radius decreasing with v so that the map is positively oriented.
    phi = 0.5 * np.pi * u
    rho = 1.0 + 0.25 * (1.0 - 2.0 * v)
    return rho * np.cos(phi), rho * np.sin(phi), 0.25 * (2.0 * w - 1.0)


def nurbs_quarter_torus(R: float = 2.0, r1: float = 0.5, r2: float = 1.0) -> Spline3D:
    """A quarter of a thick-walled torus tube, exact as a degree-2 NURBS with one element per
    direction: x = tube angle theta in [0, pi/2] (a rational quarter circle), y = radius rho in
    [r1, r2] (linear, written at degree 2), z = revolution angle phi in [0, pi/2] (a rational
    quarter circle).  The point is (d cos phi, d sin phi, rho sin theta), d = R + rho cos theta.
    Its volume is (pi/2) (R (r2^2 - r1^2) pi/4 + (r2^3 - r1^3) / 3)."""
    s = np.sqrt(0.5)
    arc = [(1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]       # quarter-circle control points on the unit circle
    warc = [1.0, s, 1.0]
    rho = [r1, 0.5 * (r1 + r2), r2]
    ctrl = np.zeros((3, 3, 3, 3))
    wts = np.zeros((3, 3, 3))
    for k in range(3):                                  # phi
        for j in range(3):                              # rho
            for i in range(3):                          # theta
                d = R + rho[j] * arc[i][0]
                z = rho[j] * arc[i][1]
                ctrl[k, j, i] = (d * arc[k][0], d * arc[k][1], z)
                wts[k, j, i] = warc[i] * warc[k]
    knots = tuple(np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0]) for _ in range(3))
    return Spline3D((2, 2, 2), knots, ctrl, wts)


def nurbs_twisted_square(length: float = 3.0) -> Spline3D:
    """A unit square section twisted by a quarter turn along an axis of the given length, exact as a
    NURBS of degrees (1, 1, 2) with one element: bilinear across the section, and along the axis the
    rational quadratic of a quarter circle (each section point travels on its own circular arc about
    the axis: control layers at 0, 45 and 90 degrees, the middle one scaled by 1 / cos 45 degrees,
    weights 1, cos 45 degrees, 1).  The twist keeps every section's area, so the volume is the length."""
    c = np.sqrt(0.5)
    ang = [0.0, 0.25 * np.pi, 0.5 * np.pi]
    scale = [1.0, 1.0 / c, 1.0]
    wz = [1.0, c, 1.0]
    ctrl = np.zeros((3, 2, 2, 3))
    wts = np.zeros((3, 2, 2))
    for k in range(3):
        ca, sa = np.cos(ang[k]), np.sin(ang[k])
        for j in range(2):
            for i in range(2):
                x, y = i - 0.5, j - 0.5
                ctrl[k, j, i] = (scale[k] * (x * ca - y * sa), scale[k] * (x * sa + y * ca), 0.5 * length * k)
                wts[k, j, i] = wz[k]
    knots = (np.array([0.0, 0.0, 1.0, 1.0]), np.array([0.0, 0.0, 1.0, 1.0]), np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0]))
    return Spline3D((1, 1, 2), knots, ctrl, wts)


def _twisted_square_nurbs(seed: int, n_boxes: int = 3, length: float = 3.0) -> Workload:
    rng = np.random.default_rng(seed)
    macro = nurbs_twisted_square(length)
    tile = identity_spline((2, 2, 2), (2, 2, 2))
    _pull_interior(tile, rng, 0.2)
    return Workload("twisted_square_nurbs", macro, tile, (1, 1, n_boxes), 1, 2, 3, 3, seed=seed)


def _twist(u, v, w):
    # a square section 1 x 1 twisted by a quarter turn along a length-3 axis
    a = 0.5 * np.pi * w
    x, y = u - 0.5, v - 0.5
    return x * np.cos(a) - y * np.sin(a), x * np.sin(a) + y * np.cos(a), 3.0 * w


def _twisted_square(seed: int, n_el: int = 2) -> Workload:
    rng = np.random.default_rng(seed)
    macro = _mapped_spline((2, 2, 2), (1, 1, 3), _twist)
    tile = identity_spline((2, 2, 2), (2, 2, 2))
    _pull_interior(tile, rng, 0.2)
    return Workload("twisted_square", macro, tile, (1, 1, 3), 0, 2, 3, 3, seed=seed)


def _nurbs_torus(seed: int, n_boxes: int = 4) -> Workload:
    rng = np.random.default_rng(seed)
    macro = nurbs_quarter_torus()
    tile = identity_spline((2, 2, 2), (3, 3, 3))
    _pull_interior(tile, rng, 0.2)
    return Workload("nurbs_torus", macro, tile, (n_boxes, n_boxes, n_boxes), 1, 2, 3, 3, seed=seed)


def family_params(seed: int, count: int) -> np.ndarray:
    """Design parameters (pinch, a_x, a_y, a_z) ~ U(0, 0.3)^4 for the parameterised tile family."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 0.3, size=(count, 4))


def tile_family(params: np.ndarray, degree: int = 2, n_el: int = 3) -> Spline3D:
    """Member of the parameterised micro-tile family.

    Interior control point i, axis k: t_ik = t0_ik + 0.5 (pinch + a_k)(0.5 - t0_ik),
    with t0 the identity (Greville) net; boundary points stay at the identity.
    """
    pinch, ax, ay, az = (float(x) for x in params)
    sp = identity_spline((degree,) * 3, (n_el,) * 3)
    mask = _interior_mask(sp.ctrl.shape[:3])
    t0 = sp.ctrl[mask]
    a = np.array([ax, ay, az])
    sp.ctrl[mask] = t0 + 0.5 * (pinch + a)[None, :] * (0.5 - t0)
    return sp


def _cfg1(seed: int) -> Workload:
    rng = np.random.default_rng(seed)
    macro = identity_spline((2, 2, 2), (2, 2, 2))
    _jitter_interior(macro, rng, 0.05)
    tile = identity_spline((2, 2, 2), (2, 2, 2))
    _pull_interior(tile, rng, 0.2)
    return Workload("cfg1", macro, tile, (2, 2, 2), 0, 2, 3, 3, seed=seed)


def _cfg2(seed: int) -> Workload:
    rng = np.random.default_rng(seed)
    macro = _mapped_spline((3, 3, 3), (16, 4, 4), _cantilever)
    _jitter_interior(macro, rng, 0.02)
    tile = identity_spline((3, 3, 3), (4, 4, 4))
    _pull_interior(tile, rng, 0.3)
    return Workload("cfg2", macro, tile, (16, 4, 4), 0, 3, 4, 3, seed=seed)


def _cfg3(seed: int, n_el: int = 32) -> Workload:
    rng = np.random.default_rng(seed)
    macro = _mapped_spline((2, 2, 2), (n_el, n_el, n_el), _torus_sector)
    tile = identity_spline((2, 2, 2), (3, 3, 3))
    _pull_interior(tile, rng, 0.2)
    return Workload("cfg3", macro, tile, (n_el, n_el, n_el), 0, 2, 3, 3, seed=seed)


def _cfg4(seed: int, n_boxes: int = 16) -> Workload:
    rng = np.random.default_rng(seed)
    macro = identity_spline((3, 3, 3), (5, 5, 5))
    _jitter_interior(macro, rng, 0.02)
    tile = identity_spline((2, 2, 2), (2, 2, 2))
    _pull_interior(tile, rng, 0.2)
    return Workload("cfg4", macro, tile, (n_boxes, n_boxes, n_boxes), 1, 3, 4, 3, seed=seed)


def _cfg5(seed: int, n_el: int = 24) -> Workload:
    macro = _mapped_spline((2, 2, 2), (n_el, n_el, n_el), _torus_sector)
    tile = tile_family(family_params(seed, 1)[0])
    w = Workload("cfg5", macro, tile, (n_el, n_el, n_el), 0, 2, 3, 3, seed=seed)
    w.extra["train_seed"] = seed + 1
    w.extra["test_seed"] = seed + 2
    w.extra["n_train"] = 512
    w.extra["n_test"] = 64
    w.extra["pod_rank"] = 64
    return w


CONFIGS = {
    "cfg1": lambda: _cfg1(1001),
    "cfg2": lambda: _cfg2(1002),
    "cfg3": lambda: _cfg3(1003),
    "cfg4": lambda: _cfg4(1004),
    "cfg5": lambda: _cfg5(1005),
}


def make(name: str, **kw) -> Workload:
    """Build a named workload.  Keyword arguments shrink the large ones for CPU-side tests:
    cfg3(n_el=...), cfg4(n_boxes=...), cfg5(n_el=...); nurbs_torus(n_boxes=...) is the exact NURBS
    quarter torus under uniform boxes; twisted_square is a square section twisted along its axis
    (a macro field far smoother across the section than along the axis), as a degree-2 B-spline;
    twisted_square_nurbs(n_boxes=...) is the exact twist as a NURBS of degrees (1, 1, 2) under
    1 x 1 x n_boxes uniform boxes."""
    seeds = {"cfg1": 1001, "cfg2": 1002, "cfg3": 1003, "cfg4": 1004, "cfg5": 1005, "nurbs_torus": 1006,
             "twisted_square": 1007, "twisted_square_nurbs": 1008}
    fn = {"cfg1": _cfg1, "cfg2": _cfg2, "cfg3": _cfg3, "cfg4": _cfg4, "cfg5": _cfg5,
          "nurbs_torus": _nurbs_torus, "twisted_square": _twisted_square,
          "twisted_square_nurbs": _twisted_square_nurbs}[name]
    return fn(seeds[name], **kw)


def affine_macro(degree: Tuple[int, int, int], n_el: Tuple[int, int, int], A: np.ndarray, b: np.ndarray) -> Spline3D:
    """Macro map x = A xi + b represented exactly as a B-spline (Greville control points mapped)."""
    sp = identity_spline(degree, n_el)
    sp.ctrl = sp.ctrl @ np.asarray(A, dtype=np.float64).T + np.asarray(b, dtype=np.float64)
    return sp


def random_displacement(n_dofs: int, seed: int) -> np.ndarray:
    """Seeded dense displacement vector (used where any u is valid, e.g. gradient checks of u^T K u)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n_dofs)
