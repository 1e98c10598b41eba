"""The linear system of the discretised elasticity problem (oracle, test infrastructure only).

Section 2.3, eq. (30): K u = f, with the stiffness matrix K (here K^pi, eq. (50)) and the load
vector f (here f^pi, eq. (53)).  Homogeneous Dirichlet conditions are imposed by removing the
clamped dofs: u = 0 there and K_ff u_f = f_f on the free dofs f.  The solution is the plain
definition, a direct sparse solve; any Krylov method applied to the same system must reach it
within its tolerance.  Section 4.2 points at Krylov methods for the large systems; which one is
not fixed there, so the oracle fixes the result, not the iteration.
"""
from __future__ import annotations

import numpy as np

from .geometry import global_grid


def face_dofs(w, face: int) -> np.ndarray:
    """Mask [n_dofs] of the dofs of the control points on macro face `face` = 2 d + side
    (side 0: global index 0 along d, side 1: the last)."""
    d, side = divmod(face, 2)
    G = global_grid(w)
    idx = np.indices((G[2], G[1], G[0]))          # z, y, x; G = x + GX (y + GY z)
    along = {0: idx[2], 1: idx[1], 2: idx[0]}[d].reshape(-1)
    on = along == (G[d] - 1 if side else 0)
    return np.repeat(on, 3)


def dirichlet_solve(row_ptr, col_idx, vals, f: np.ndarray, fixed: np.ndarray) -> np.ndarray:
    """u with u[fixed] = 0 and (K u - f)[free] = 0 (direct sparse LU of K_ff)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    n = len(row_ptr) - 1
    K = sp.csr_matrix((vals, col_idx.astype(np.int64), row_ptr), shape=(n, n))
    free = ~np.asarray(fixed, bool)
    u = np.zeros(n)
    u[free] = spl.spsolve(K[free][:, free].tocsc(), f[free])
    return u
