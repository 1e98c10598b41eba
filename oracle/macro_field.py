"""Macro fields of the internal work (oracle, test infrastructure only).

The paper's curvilinear route (Appendix A.1-A.2):
  covariant basis       g_i = M^(t)_{,xi_i}                      eq. (79)
  covariant metric      g_ij = g_i . g_j, contravariant = inverse eq. (81)
  material tensor       C^ijkl = lam g^ij g^kl + mu (g^ik g^jl + g^il g^jk)   eq. (84a)
  Voigt order           (11, 22, 33, 23, 13, 12)                  eq. (90), (93)
  strain blocks         G_1 = [g1 0 0 0 g3 g2], G_2 = [0 g2 0 g3 0 g1],
                        G_3 = [0 0 g3 g2 g1 0]                    eq. (91)
  macro field           A_ij = G_i C G_j^T |det J_M|              eq. (37), (97)

``cartesian_field`` is an independent second formula for the same quantity,
obtained from the Cartesian form sigma:eps = lam div u div v + mu (grad u : grad v
+ grad u : grad v^T) after the change of variables x = M(xi); it is used only to
pin the curvilinear route.
"""
from __future__ import annotations

import numpy as np

VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def lame(E: float, nu: float):
    """Lame constants (lambda, mu) of an isotropic 3-D material from E and nu."""
    return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def _Gblocks(g):
    """The three 3x6 strain blocks of eq. (91) from the covariant vectors g[..., :, i] = g_i."""
    shp = g.shape[:-2]
    G = np.zeros(shp + (3, 3, 6), dtype=g.dtype)  # G[..., i, row, voigt]
    g1, g2, g3 = g[..., :, 0], g[..., :, 1], g[..., :, 2]
    G[..., 0, :, 0] = g1
    G[..., 0, :, 4] = g3
    G[..., 0, :, 5] = g2
    G[..., 1, :, 1] = g2
    G[..., 1, :, 3] = g3
    G[..., 1, :, 5] = g1
    G[..., 2, :, 2] = g3
    G[..., 2, :, 3] = g2
    G[..., 2, :, 4] = g1
    return G


def contravariant_material(g, lam, mu):
    """Voigt 6x6 matrix of eq. (93) built from eq. (81) and (84a)."""
    gcov = np.einsum("...ci,...cj->...ij", g, g)
    gcon = np.linalg.inv(gcov)
    shp = g.shape[:-2]
    C = np.zeros(shp + (6, 6), dtype=g.dtype)
    for I, (i, j) in enumerate(VOIGT):
        for K, (k, l) in enumerate(VOIGT):
            C[..., I, K] = lam * gcon[..., i, j] * gcon[..., k, l] + mu * (
                gcon[..., i, k] * gcon[..., j, l] + gcon[..., i, l] * gcon[..., j, k])
    return C


def macro_field(J, lam, mu, signed_det: bool = False):
    """A_ij (shape (..., 3, 3, 3, 3) indexed [i, j, a, b]) from the macro-element Jacobian J.

    J[..., c, i] = d M^(t)_c / d xi_i, i.e. column i is the covariant vector g_i (eq. (79)).
    |det J| per eq. (37); with signed_det the determinant itself is used (analytic in J,
    needed only for complex-step differentiation, valid where det J > 0).
    """
    C = contravariant_material(J, lam, mu)
    G = _Gblocks(J)
    det = np.linalg.det(J)
    D = det if signed_det else np.abs(det)
    A = np.einsum("...iar,...rs,...jbs->...ijab", G, C, G)
    return A * D[..., None, None, None, None]


def cartesian_field(J, lam, mu):
    """Independent Cartesian form of the same field: with F = J^-1 and F_i its i-th row,
    A_ij,ab = det J [lam F_ia F_jb + mu (F_i . F_j) delta_ab + mu F_ib F_ja]."""
    F = np.linalg.inv(J)
    D = np.abs(np.linalg.det(J))
    eye = np.eye(3)
    A = (lam * np.einsum("...ia,...jb->...ijab", F, F)
         + mu * np.einsum("...ik,...jk->...ij", F, F)[..., None, None] * eye
         + mu * np.einsum("...ib,...ja->...ijab", F, F))
    return A * D[..., None, None, None, None]
