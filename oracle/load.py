"""Load vector f^pi of the multiscale assembly (oracle, test infrastructure only).

Section 3.2.2-3.2.3 and Appendix A.1:
* body term: bbar(xi) = b |det J_M^(t)(xi)| on the tile's box coordinates xi in [0,1]^3
  (eq. (40), (86); J_M^(t) includes the box scaling diag(h)), projected onto the
  Bernstein space Q_q as the stiffness field (eq. (44), with the operator of eq. (23)-(24));
* traction term on macro face F (xi_d = 0 or 1): tbar_F(xi) = t_F |det I_M^(t)|, which for a
  face xi_d = const is the area element |d_u M^(t) x d_v M^(t)| (eq. (41), (87)-(88));
  projected onto the face's Bernstein functions N_C, C in I_F (those with c_d = 0 on xi_d = 0,
  c_d = q on xi_d = 1), by the face's own (q+1)^2 system (eq. (45));
* table (eq. (54)-(55)), pulled back to the tile parameter domain:
    F[A, C, 0]     = int_[0,1]^3 R_A(theta) N_C(T^r(theta)) det J_T(theta) dtheta,
    F[A, C, 1 + f] = int over tile face f of R_A(theta) N_C(theta) dGamma
  (the tile's boundary control points sit at the identity positions, so T^r is the identity on
  its faces and dGamma is the unit-square measure); faces f = 2 d + side, side 0: theta_d = 0;
* tile vectors (eq. (53)): f^(t)[A, a] = sum_C <bbar_a>_C F[A, C, 0]
                                       + sum_{f touched} sum_{C in I_f} <tbar_f,a>_C F[A, C, 1 + f];
* global vector: f[3 G + a] = sum over the tiles holding G, in ascending tile index.

A tile touches macro face f (direction d, side s) when its box does: tile index 0 (s = 0) or
tiles_d - 1 (s = 1) along d.  b and t_f are constant vectors in physical space.
"""
from __future__ import annotations

import numpy as np

from .basis import bernstein, bspline_basis, gauss01
from .geometry import (eval_volume_grid, eval_volume_points, n_global_dofs, tile_boxes, tile_global_indices,
                       tile_index)
from .projection import bernstein3, degrees, fit_points, n_pi, projection_operator
from .tables import active_functions, element_points, micro_elements

N_FACES = 6


def face_axes(f: int):
    """(d, side, u, v) of face f = 2 d + side: the normal direction, the side, the in-face axes."""
    d, side = divmod(f, 2)
    u, v = [k for k in range(3) if k != d]
    return d, side, u, v


def face_index_set(q, f: int) -> np.ndarray:
    """I_f: the Bernstein indices C = c1 + (q1+1)(c2 + (q2+1) c3) that do not vanish on face f
    (q an int or a degree triple)."""
    d, side, _, _ = face_axes(f)
    qd = degrees(q)
    out = []
    for C in range(n_pi(q)):
        c = (C % (qd[0] + 1), (C // (qd[0] + 1)) % (qd[1] + 1), C // ((qd[0] + 1) * (qd[1] + 1)))
        if c[d] == (qd[d] if side else 0):
            out.append(C)
    return np.array(out, dtype=np.int64)


def face_projection_operator(q, n_fit: int) -> np.ndarray:
    """2-D version of eq. (23)-(24) on [0,1]^2 with degrees q = (q_u, q_v) (or one int):
    P2 ((q_u+1)(q_v+1) x n_fit^2), index c_u + (q_u+1) c_v, point s_u + n_fit s_v."""
    qu, qv = (int(q), int(q)) if np.ndim(q) == 0 else (int(q[0]), int(q[1]))
    x, wx = gauss01(n_fit)
    Bu, Bv = bernstein(qu, x), bernstein(qv, x)            # (n_fit, q+1)
    N = np.einsum("vj,ui->vuji", Bv, Bu).reshape(n_fit * n_fit, -1)   # [(s_v, s_u), (c_v, c_u)]
    W = np.einsum("v,u->vu", wx, wx).reshape(-1)
    M = N.T @ (W[:, None] * N)
    return np.linalg.solve(M, N.T * W[None, :])


def load_table(tile, q, n_g: int) -> np.ndarray:
    """F of eq. (54)-(55): shape (n_T, n_pi, 7), slot 0 the volume, 1 + f the faces."""
    nT = int(np.prod(tile.n_ctrl))
    npi = n_pi(q)
    F = np.zeros((nT, npi, 1 + N_FACES))
    # volume: micro elements and their Gauss points
    for e, box in micro_elements(tile):
        act = np.array(active_functions(tile, e))
        R, _, X, J, w = element_points(tile, box, n_g)
        det = np.linalg.det(J)
        N = bernstein3(q, X)                                       # (G, n_pi)
        F[act, :, 0] += np.einsum("g,gA,gC->AC", w * det, R[:, act], N)
    # faces: the micro element faces on the tile face, 2-D Gauss points, identity map on the face
    xg, wg = gauss01(n_g)
    n = tile.n_ctrl
    for f in range(N_FACES):
        d, side, u, v = face_axes(f)
        knots_u, knots_v = tile.knots[u], tile.knots[v]
        spans_u = [(knots_u[i], knots_u[i + 1]) for i in range(len(knots_u) - 1) if knots_u[i + 1] > knots_u[i]]
        spans_v = [(knots_v[i], knots_v[i + 1]) for i in range(len(knots_v) - 1) if knots_v[i + 1] > knots_v[i]]
        Nd = bspline_basis(tile.knots[d], tile.degree[d], np.array([float(side)]))[0]   # (n_d,)
        for (lu, hu) in spans_u:
            for (lv, hv) in spans_v:
                pu, pv = lu + (hu - lu) * xg, lv + (hv - lv) * xg
                Nu = bspline_basis(knots_u, tile.degree[u], pu)         # (n_g, n_u)
                Nv = bspline_basis(knots_v, tile.degree[v], pv)
                wu, wv = (hu - lu) * wg, (hv - lv) * wg
                # face points (s_v, s_u) and their xi = theta on the face
                th = np.zeros((n_g * n_g, 3))
                PV, PU = np.meshgrid(pv, pu, indexing="ij")
                th[:, d] = side
                th[:, u] = PU.ravel()
                th[:, v] = PV.ravel()
                NC = bernstein3(q, th)                                  # (n_g^2, n_pi)
                wt = np.einsum("v,u->vu", wv, wu).ravel()
                # R_A on the face: product of the 1-D bases, A = i + n_x (j + n_y k)
                Rf = np.zeros((n_g * n_g, nT))
                for k3 in range(n[2]):
                    for k2 in range(n[1]):
                        for k1 in range(n[0]):
                            idx = (k1, k2, k3)
                            val = Nd[idx[d]] * np.einsum("v,u->vu", Nv[:, idx[v]], Nu[:, idx[u]]).ravel()
                            Rf[:, k1 + n[0] * (k2 + n[1] * k3)] = val
                F[:, :, 1 + f] += np.einsum("g,gA,gC->AC", wt, Rf, NC)
    return F


def _box(w, t):
    boxes = tile_boxes(w)
    tx, ty, tz = tile_index(w, t)
    a = np.array([boxes[0][0][tx], boxes[1][0][ty], boxes[2][0][tz]])
    h = np.array([boxes[0][1][tx], boxes[1][1][ty], boxes[2][1][tz]])
    return a, h, (tx, ty, tz)


def touched_faces(w, t: int):
    """Macro faces f (2 d + side) that tile t's box touches."""
    _, _, ti = _box(w, t)
    out = []
    for d in range(3):
        if ti[d] == 0:
            out.append(2 * d)
        if ti[d] == w.tiles[d] - 1:
            out.append(2 * d + 1)
    return out


def load_coefficients(w, t: int, body, traction, P=None, P2=None) -> np.ndarray:
    """Projection coefficients of tile t, shape (7, 3, n_pi): slot 0 <bbar>, slot 1 + f <tbar_f> on I_f."""
    body = np.asarray(body, dtype=np.float64)
    traction = np.asarray(traction, dtype=np.float64).reshape(N_FACES, 3)
    q, nf = w.q, w.n_fit
    qd = degrees(q)
    npi = n_pi(q)
    P = projection_operator(q, nf) if P is None else P
    a, h, _ = _box(w, t)
    out = np.zeros((1 + N_FACES, 3, npi))
    # body: samples at the tensor GL nodes (x fastest), |det J_M^(t)|
    x, _ = gauss01(nf)
    _, J = eval_volume_grid(w.macro.degree, w.macro.knots, w.macro.ctrl, a[0] + h[0] * x, a[1] + h[1] * x,
                            a[2] + h[2] * x, weights=w.macro.weights)
    det = np.abs(np.linalg.det(J.reshape(-1, 3, 3) * h[None, None, :]))
    out[0] = (P @ (det[:, None] * body[None, :])).T
    # tractions on the touched macro faces
    for f in touched_faces(w, t):
        d, side, u, v = face_axes(f)
        pts = np.zeros((nf * nf, 3))
        PV, PU = np.meshgrid(x, x, indexing="ij")
        pts[:, d] = side
        pts[:, u] = PU.ravel()
        pts[:, v] = PV.ravel()
        _, Jp = eval_volume_points(w.macro.degree, w.macro.knots, w.macro.ctrl, a + h * pts, weights=w.macro.weights)
        Jp = Jp * h[None, None, :]
        area = np.linalg.norm(np.cross(Jp[:, :, u], Jp[:, :, v]), axis=1)
        P2f = P2 if (P2 is not None and qd[u] == qd[v]) else face_projection_operator((qd[u], qd[v]), nf)
        cf = P2f @ (area[:, None] * traction[f][None, :])             # index c_u + (q_u+1) c_v
        for cv in range(qd[v] + 1):
            for cu in range(qd[u] + 1):
                c = [0, 0, 0]
                c[d] = qd[d] if side else 0
                c[u], c[v] = cu, cv
                C = c[0] + (qd[0] + 1) * (c[1] + (qd[1] + 1) * c[2])
                out[1 + f, :, C] = cf[cu + (qd[u] + 1) * cv]
    return out


def tile_load(table: np.ndarray, coef: np.ndarray) -> np.ndarray:
    """f^(t) of eq. (53): (n_T, 3) from the table (n_T, n_pi, 7) and the coefficients (7, 3, n_pi)."""
    return np.einsum("ACs,saC->Aa", table, coef)


def assemble_load(w, table, body, traction) -> np.ndarray:
    """Global f^pi [3 N_G]: tile vectors summed over the tiles holding each point, in ascending tile order."""
    f = np.zeros(n_global_dofs(w))
    P = projection_operator(w.q, w.n_fit)
    P2 = face_projection_operator(w.q, w.n_fit) if np.ndim(w.q) == 0 else None
    for t in range(w.n_tiles):
        ft = tile_load(table, load_coefficients(w, t, body, traction, P, P2))
        G = tile_global_indices(w, t)
        for a in range(3):
            np.add.at(f, 3 * G + a, ft[:, a])
    return f


def standard_load(w, body, traction, n_g: int = None) -> np.ndarray:
    """f^bullet by Gauss quadrature of the composed map (no projection, no table), for eq. (63):
    f[3 G_A + a] += int R_A b_a dx + sum over the macro faces int R_A t_a dGamma."""
    n_g = w.n_gauss if n_g is None else n_g
    body = np.asarray(body, dtype=np.float64)
    traction = np.asarray(traction, dtype=np.float64).reshape(N_FACES, 3)
    f = np.zeros(n_global_dofs(w))
    tile = w.tile
    nT = int(np.prod(tile.n_ctrl))
    n = tile.n_ctrl
    xg, wg = gauss01(n_g)
    for t in range(w.n_tiles):
        a, h, _ = _box(w, t)
        G = tile_global_indices(w, t)
        ft = np.zeros((nT, 3))
        for e, box in micro_elements(tile):
            act = np.array(active_functions(tile, e))
            R, _, X, JT, wts = element_points(tile, box, n_g)
            _, JM = eval_volume_points(w.macro.degree, w.macro.knots, w.macro.ctrl, a + h * X, weights=w.macro.weights)
            J = (JM * h[None, None, :]) @ JT
            det = np.abs(np.linalg.det(J))
            ft[act] += np.einsum("g,gA->A", wts * det, R[:, act])[:, None] * body[None, :]
        for f_ in touched_faces(w, t):
            d, side, u, v = face_axes(f_)
            spans_u = [(tile.knots[u][i], tile.knots[u][i + 1]) for i in range(len(tile.knots[u]) - 1)
                       if tile.knots[u][i + 1] > tile.knots[u][i]]
            spans_v = [(tile.knots[v][i], tile.knots[v][i + 1]) for i in range(len(tile.knots[v]) - 1)
                       if tile.knots[v][i + 1] > tile.knots[v][i]]
            for (lu, hu) in spans_u:
                for (lv, hv) in spans_v:
                    pu, pv = lu + (hu - lu) * xg, lv + (hv - lv) * xg
                    th = np.zeros((n_g * n_g, 3))
                    PV, PU = np.meshgrid(pv, pu, indexing="ij")
                    th[:, d] = side
                    th[:, u] = PU.ravel()
                    th[:, v] = PV.ravel()
                    Bx, dBx = bspline_basis(tile.knots[0], tile.degree[0], th[:, 0], deriv=True)
                    By, dBy = bspline_basis(tile.knots[1], tile.degree[1], th[:, 1], deriv=True)
                    Bz, dBz = bspline_basis(tile.knots[2], tile.degree[2], th[:, 2], deriv=True)
                    R = np.einsum("pk,pj,pi->pkji", Bz, By, Bx).reshape(len(th), -1)
                    dR = np.stack([np.einsum("pk,pj,pi->pkji", Bz, By, dBx).reshape(len(th), -1),
                                   np.einsum("pk,pj,pi->pkji", Bz, dBy, Bx).reshape(len(th), -1),
                                   np.einsum("pk,pj,pi->pkji", dBz, By, Bx).reshape(len(th), -1)], axis=-1)
                    ctrl = tile.ctrl.reshape(-1, 3)
                    X = R @ ctrl
                    JT = np.einsum("gAk,Ac->gck", dR, ctrl)
                    _, JM = eval_volume_points(w.macro.degree, w.macro.knots, w.macro.ctrl, a + h * X, weights=w.macro.weights)
                    J = (JM * h[None, None, :]) @ JT
                    area = np.linalg.norm(np.cross(J[:, :, u], J[:, :, v]), axis=1)
                    wt = np.einsum("v,u->vu", (hv - lv) * wg, (hu - lu) * wg).ravel()
                    ft += np.einsum("g,gA->A", wt * area, R)[:, None] * traction[f_][None, :]
        for c in range(3):
            np.add.at(f, 3 * G + c, ft[:, c])
    return f


def _abs_det(J):
    """|det J| of (S, 3, 3) Jacobians, continued analytically for the complex step: the sign of the
    real part's determinant times the (complex) determinant."""
    d = np.linalg.det(J)
    return np.sign(np.linalg.det(J.real)) * d


def _face_area(J, u, v):
    """|J e_u x J e_v| of (S, 3, 3) Jacobians as sqrt(n . n) (analytic in J for the complex step)."""
    n = np.cross(J[:, :, u], J[:, :, v])
    return np.sqrt(np.sum(n * n, axis=1))


def _complex_step_grad(fun, J, h=1e-30):
    """d fun(J)/dJ_mn for a scalar-per-sample function of (S, 3, 3) Jacobians, shape (S, 3, 3)."""
    out = np.empty(J.shape)
    for m in range(3):
        for n in range(3):
            Jc = J.astype(np.complex128)
            Jc[:, m, n] += 1j * h
            out[:, m, n] = fun(Jc).imag / h
    return out


def uf(w, table, body, traction, u) -> float:
    """u . f^pi as the sum of the tile terms u^(t) . f^(t) (eq. (53) glued)."""
    P = projection_operator(w.q, w.n_fit)
    total = 0.0
    for t in range(w.n_tiles):
        ut = u[3 * tile_global_indices(w, t)[:, None] + np.arange(3)[None, :]]
        total += float(np.sum(ut * tile_load(table, load_coefficients(w, t, body, traction, P))))
    return total


def grad_uf(w, table, body, traction, u) -> np.ndarray:
    """d(u . f^pi)/dm for a fixed vector u, shape like w.macro.ctrl (NURBS: weights fixed).

    The external work of eq. (69) differentiated through its projections (eq. (40)-(41), (44)-(45)):
    per tile, Y[slot, a, C] = sum_A u_(A,a) F[A, C, slot] is the adjoint of the lookup (eq. (53));
    the projection's transpose gives the adjoint of the sampled fields, d(u.f)/d|det J_s| and
    d(u.f)/d area_s; the derivatives of |det J| and of the face area element by J come from a
    complex step of their definitions (no hand-derived formula); J = J_M(a + h xi) diag(h) gives
    dJ/dm_k,c = e_c (grad N_k * h)^T, summed over the sample grids as for the stiffness gradient."""
    from .geometry import control_point_gradient
    body = np.asarray(body, dtype=np.float64)
    traction = np.asarray(traction, dtype=np.float64).reshape(N_FACES, 3)
    qd = degrees(w.q)
    P = projection_operator(w.q, w.n_fit)
    x, _ = gauss01(w.n_fit)
    nf = len(x)
    wts = getattr(w.macro, "weights", None)
    g = np.zeros_like(w.macro.ctrl)
    for t in range(w.n_tiles):
        a, h, _ = _box(w, t)
        ut = u[3 * tile_global_indices(w, t)[:, None] + np.arange(3)[None, :]]   # (n_T, 3)
        Y = np.einsum("Aa,ACs->saC", ut, table)                                     # (7, 3, n_pi)
        # body: coef[0][a][C] = b_a sum_s P[C, s] |det J_s|
        gbar = P.T @ (body @ Y[0])                                                  # (S,)
        _, JM = eval_volume_grid(w.macro.degree, w.macro.knots, w.macro.ctrl, a[0] + h[0] * x, a[1] + h[1] * x,
                                 a[2] + h[2] * x, weights=wts)
        J = JM.reshape(-1, 3, 3) * h[None, None, :]
        Jbar = gbar[:, None, None] * _complex_step_grad(_abs_det, J) * h[None, None, :]
        g += control_point_gradient(w.macro.knots, w.macro.degree, wts, a[0] + h[0] * x, a[1] + h[1] * x,
                                    a[2] + h[2] * x, Jbar.reshape(nf, nf, nf, 3, 3))
        for f in touched_faces(w, t):
            d, side, uu, vv = face_axes(f)
            P2f = face_projection_operator((qd[uu], qd[vv]), nf)                    # [(c_u, c_v), (s_v, s_u)]
            ybar = np.zeros(P2f.shape[0])
            for cv in range(qd[vv] + 1):
                for cu in range(qd[uu] + 1):
                    c = [0, 0, 0]
                    c[d] = qd[d] if side else 0
                    c[uu], c[vv] = cu, cv
                    C = c[0] + (qd[0] + 1) * (c[1] + (qd[1] + 1) * c[2])
                    ybar[cu + (qd[uu] + 1) * cv] = traction[f] @ Y[1 + f, :, C]
            abar = P2f.T @ ybar                                                     # (nf^2,) s = s_u + nf s_v
            pts = np.zeros((nf * nf, 3))
            PV, PU = np.meshgrid(x, x, indexing="ij")
            pts[:, d] = side
            pts[:, uu] = PU.ravel()
            pts[:, vv] = PV.ravel()
            _, Jp = eval_volume_points(w.macro.degree, w.macro.knots, w.macro.ctrl, a + h * pts, weights=wts)
            Jp = Jp * h[None, None, :]
            Jbar = abar[:, None, None] * _complex_step_grad(lambda Jc: _face_area(Jc, uu, vv), Jp) * h[None, None, :]
            # the face grid as (z, y, x) with one point along d; v is the slower in-face axis
            shape = [nf, nf, nf]
            shape[2 - d] = 1
            axes = [a[k] + h[k] * (x if k != d else np.array([float(side)])) for k in range(3)]
            g += control_point_gradient(w.macro.knots, w.macro.degree, wts, axes[0], axes[1], axes[2],
                                        Jbar.reshape(shape[0], shape[1], shape[2], 3, 3))
    return g
