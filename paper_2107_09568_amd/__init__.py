"""igamt: interpolation-and-lookup assembly of isogeometric stiffness matrices of
microstructured (spline-composed) geometries on AMD MI355X.

Python binding of libigamt (include/igamt.h).  This layer only marshals
arguments: host arrays become plain pointers, device buffers are torch CUDA
tensors (HIP memory) and the stream is torch's current HIP stream.  Every step
of the computation runs in the library's HIP kernels; the binding raises if
the library is missing.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Tuple

import numpy as np

from . import _lib
from ._lib import IgamtError, check, lib

F64, F32, BF16X3, F16X3 = 0, 1, 2, 3
PRECISIONS = {"f64": F64, "f32": F32, "bf16x3": BF16X3, "f16x3": F16X3}

__all__ = ["Plan", "F64", "F32", "BF16X3", "F16X3", "PRECISIONS", "IgamtError", "spmv", "lib"]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _spline(degree, knots, ctrl, keep, weights=None):
    s = _lib.Spline3D()
    ctrl = np.ascontiguousarray(ctrl, dtype=np.float64)
    ks = [np.ascontiguousarray(k, dtype=np.float64) for k in knots]
    keep.extend([ctrl] + ks)
    if weights is not None:
        weights = np.ascontiguousarray(weights, dtype=np.float64)
        assert weights.shape == ctrl.shape[:3], "one weight per control point"
        keep.append(weights)
        s.weights = weights.ctypes.data_as(_lib.P_f64)
    for d in range(3):
        s.degree[d] = int(degree[d])
        s.knots[d] = ks[d].ctypes.data_as(_lib.P_f64)
    s.n_ctrl[0], s.n_ctrl[1], s.n_ctrl[2] = ctrl.shape[2], ctrl.shape[1], ctrl.shape[0]
    s.ctrl = ctrl.ctypes.data_as(_lib.P_f64)
    return s


class Plan:
    """A fixed topology: macro map, reference tile, tile grid, projection degree.

    macro, tile: objects with .degree (3 ints), .knots (3 arrays), .ctrl ((nz, ny, nx, 3) array).
    """

    def __init__(self, macro, tile, tiles, box_mode=0, q=2, n_fit=None, n_gauss=3):
        keep = []
        m = _spline(macro.degree, macro.knots, macro.ctrl, keep, getattr(macro, "weights", None))
        t = _spline(tile.degree, tile.knots, tile.ctrl, keep, getattr(tile, "weights", None))
        d = _lib.PlanDesc()
        for k in range(3):
            d.tiles[k] = int(tiles[k])
        d.box_mode = int(box_mode)
        qd = (int(q),) * 3 if np.ndim(q) == 0 else tuple(int(v) for v in q)
        d.q = max(qd)
        d.anisotropic = int(np.ndim(q) != 0)
        for k in range(3):
            d.q_dir[k] = qd[k]
        d.n_fit = int(max(qd) + 1 if n_fit is None else n_fit)
        d.n_gauss = int(n_gauss)
        h = C.c_void_p()
        check(lib().igamt_plan_create(C.byref(m), C.byref(t), C.byref(d), C.byref(h)))
        self._h = h
        self.macro_ctrl_shape = np.asarray(macro.ctrl).shape
        self.tile_ctrl_shape = np.asarray(tile.ctrl).shape
        nz, ny, nx = self.tile_ctrl_shape[:3]
        self.grid = tuple(int(tiles[k]) * (n - 1) + 1 for k, n in enumerate((nx, ny, nz)))   # global ctrl, x y z
        s = _lib.Sizes()
        check(lib().igamt_plan_sizes(h, C.byref(s)))
        self.sizes = {f: getattr(s, f) for f, _ in _lib.Sizes._fields_}
        self.q_dir = qd                     # projection degrees per direction
        self.q = max(qd)

    @classmethod
    def from_workload(cls, w):
        return cls(w.macro, w.tile, w.tiles, w.box_mode, w.q, w.n_fit, w.n_gauss)

    def close(self):
        if getattr(self, "_h", None):
            lib().igamt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __getattr__(self, name):
        sizes = self.__dict__.get("sizes")
        if sizes is not None and name in sizes:
            return sizes[name]
        raise AttributeError(name)

    # ---- host integer set-up ----------------------------------------------------
    def pairs(self) -> np.ndarray:
        out = np.empty((self.n_pairs, 2), dtype=np.int32)
        check(lib().igamt_plan_pairs(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def csr_host(self) -> Tuple[np.ndarray, np.ndarray]:
        rp = np.empty(self.n_dofs + 1, dtype=np.int64)
        ci = np.empty(self.nnz, dtype=np.int32)
        check(lib().igamt_plan_csr(self._h, rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p)))
        return rp, ci

    # ---- device ---------------------------------------------------------------------
    def csr_device(self):
        torch = _torch()
        rp = torch.empty(self.n_dofs + 1, dtype=torch.int64, device="cuda")
        ci = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        check(lib().igamt_plan_csr_device(self._h, _ptr(rp), _ptr(ci), _stream()))
        return rp, ci

    def set_macro_ctrl(self, ctrl):
        torch = _torch()
        if isinstance(ctrl, torch.Tensor):
            assert ctrl.is_cuda and ctrl.dtype == torch.float64 and ctrl.is_contiguous()
            assert ctrl.numel() == 3 * self.n_macro_ctrl
            check(lib().igamt_set_macro_ctrl(self._h, _ptr(ctrl), 1, _stream()))
        else:
            a = np.ascontiguousarray(ctrl, dtype=np.float64)
            assert a.size == 3 * self.n_macro_ctrl
            check(lib().igamt_set_macro_ctrl(self._h, a.ctypes.data_as(C.c_void_p), 0, _stream()))

    def set_tile_ctrl(self, ctrl):
        torch = _torch()
        if isinstance(ctrl, torch.Tensor):
            assert ctrl.is_cuda and ctrl.dtype == torch.float64 and ctrl.is_contiguous()
            assert ctrl.numel() == 3 * self.n_tile_ctrl
            check(lib().igamt_set_tile_ctrl_device(self._h, _ptr(ctrl), _stream()))
        else:
            a = np.ascontiguousarray(ctrl, dtype=np.float64)
            assert a.size == 3 * self.n_tile_ctrl
            check(lib().igamt_set_tile_ctrl(self._h, a.ctypes.data_as(C.c_void_p)))

    def tables_build(self, gate=None):
        if gate is None:
            check(lib().igamt_tables_build(self._h, _stream()))
        else:
            torch = _torch()
            assert gate.is_cuda and gate.dtype == torch.int32
            check(lib().igamt_tables_build_gated(self._h, _ptr(gate), _stream()))

    def tables_set(self, table):
        torch = _torch()
        assert table.is_cuda and table.dtype == torch.float64 and table.shape == (self.n_pairs, self.n_cols)
        table = table.contiguous()
        check(lib().igamt_tables_set(self._h, _ptr(table), _stream()))

    def tables_get(self):
        torch = _torch()
        out = torch.empty((self.n_pairs, self.n_cols), dtype=torch.float64, device="cuda")
        check(lib().igamt_tables_get(self._h, _ptr(out), _stream()))
        return out

    def tables_build_rows(self, rows):
        torch = _torch()
        rows = rows.to(device="cuda", dtype=torch.int32).contiguous()
        out = torch.empty((rows.numel(), self.n_cols), dtype=torch.float64, device="cuda")
        check(lib().igamt_tables_build_rows(self._h, _ptr(rows), int(rows.numel()), _ptr(out), _stream()))
        return out

    def workspace_bytes(self, prec):
        cb, bb = C.c_int64(), C.c_int64()
        check(lib().igamt_workspace_bytes(self._h, _prec(prec), C.byref(cb), C.byref(bb)))
        return cb.value, bb.value

    def _empty_bytes(self, nbytes):
        torch = _torch()
        return torch.empty(max(int(nbytes), 256) // 8 + 1, dtype=torch.float64, device="cuda")

    def fit(self, E, nu, prec="f64", out=None):
        cb, _ = self.workspace_bytes(prec)
        out = self._empty_bytes(cb) if out is None else out
        check(lib().igamt_fit(self._h, float(E), float(nu), _prec(prec), _ptr(out), _stream()))
        return out

    def coef_view(self, coef, prec="f64"):
        """Fitted coefficients as (n_tiles, K, 9) float64 for inspection (F64/F32 modes only)."""
        torch = _torch()
        p = _prec(prec)
        npad, Kp, K = self.n_tiles_pad, self.n_cols_pad, self.n_cols
        if p == F64:
            v = coef.view(torch.float64)[: npad * 9 * Kp]
        elif p == F32:
            v = coef.view(torch.float32)[: npad * 9 * Kp].double()
        else:
            raise ValueError("coefficient view only for f64 / f32")
        return v.view(npad, 9, Kp)[: self.n_tiles, :, :K].transpose(1, 2)

    def contract(self, coef, prec="f64", out=None):
        torch = _torch()
        dt = torch.float64 if _prec(prec) == F64 else torch.float32
        out = torch.empty((self.n_tiles, self.n_pairs, 9), dtype=dt, device="cuda") if out is None else out
        check(lib().igamt_contract(self._h, _prec(prec), _ptr(coef), _ptr(out), _stream()))
        return out

    def contract_products(self, coef, products, out=None):
        """Ablations of the BF16 split contraction on BF16X3 coefficients: products = 2 (table split
        only), 3 (the split mode) or 4 (with lo*lo); FP32 blocks [n_tiles, n_pairs, 9]."""
        torch = _torch()
        if out is None:
            out = torch.empty((self.n_tiles, self.n_pairs, 9), dtype=torch.float32, device="cuda")
        check(lib().igamt_contract_products(self._h, int(products), _ptr(coef), _ptr(out), _stream()))
        return out

    def scatter(self, blocks, prec="f64", out=None):
        torch = _torch()
        dt = torch.float64 if _prec(prec) == F64 else torch.float32
        out = torch.empty(self.nnz, dtype=dt, device="cuda") if out is None else out
        check(lib().igamt_scatter(self._h, _prec(prec), _ptr(blocks), _ptr(out), _stream()))
        return out

    def workspace(self, prec):
        cb, bb = self.workspace_bytes(prec)
        return self._empty_bytes(cb + bb)

    def assemble(self, E, nu, prec="f64", values=None, workspace=None):
        torch = _torch()
        dt = torch.float64 if _prec(prec) == F64 else torch.float32
        values = torch.empty(self.nnz, dtype=dt, device="cuda") if values is None else values
        workspace = self.workspace(prec) if workspace is None else workspace
        check(lib().igamt_assemble(self._h, float(E), float(nu), _prec(prec), _ptr(values), _ptr(workspace),
                                   _stream()))
        return values

    def check(self):
        bad = C.c_int64()
        code = lib().igamt_check(self._h, _stream(), C.byref(bad))
        if code != 0:
            raise IgamtError(code, lib().igamt_last_error().decode())

    # ---- sensitivities ------------------------------------------------------------
    def grad_workspace(self, prec):
        b = C.c_int64()
        check(lib().igamt_grad_workspace_bytes(self._h, _prec(prec), C.byref(b)))
        return self._empty_bytes(b.value)

    def uKu_grad(self, E, nu, u, prec="f64", workspace=None):
        """(u^T K u, d(u^T K u)/d macro control points) with u fixed."""
        torch = _torch()
        assert u.is_cuda and u.dtype == torch.float64 and u.numel() == self.n_dofs
        u = u.contiguous()
        grad = torch.empty(self.macro_ctrl_shape, dtype=torch.float64, device="cuda")
        val = torch.empty(1, dtype=torch.float64, device="cuda")
        ws = self.grad_workspace(prec) if workspace is None else workspace
        check(lib().igamt_uKu_grad(self._h, float(E), float(nu), _prec(prec), _ptr(u), _ptr(grad), _ptr(val),
                                   _ptr(ws), _stream()))
        return val, grad

    # ---- learned tables ------------------------------------------------------------------
    def table_from_pod(self, mean, basis, coeffs, scale=1.0):
        r = basis.shape[0]
        check(lib().igamt_table_from_pod(self._h, _ptr(mean), _ptr(basis), int(r), _ptr(coeffs.contiguous()),
                                         float(scale), _stream()))

    def table_rows_check(self, rows, exact_rows, tol, err=None, gate=None):
        """(relative error on the rows, int32 gate = error > tol), both left on the device."""
        torch = _torch()
        err = torch.empty(1, dtype=torch.float64, device="cuda") if err is None else err
        gate = torch.empty(1, dtype=torch.int32, device="cuda") if gate is None else gate
        check(lib().igamt_table_rows_check(self._h, _ptr(rows), int(rows.numel()), _ptr(exact_rows), float(tol),
                                           _ptr(err), _ptr(gate), _stream()))
        return err, gate

    def table_rows_error(self, rows, exact_rows):
        torch = _torch()
        err = torch.empty(1, dtype=torch.float64, device="cuda")
        rows = rows.to(device="cuda", dtype=torch.int32).contiguous()
        check(lib().igamt_table_rows_error(self._h, _ptr(rows), int(rows.numel()), _ptr(exact_rows), _ptr(err),
                                           _stream()))
        return err

    # ---- load vector ----------------------------------------------------------------------
    @staticmethod
    def _loads(body, traction):
        b = np.ascontiguousarray(body, dtype=np.float64).reshape(3)
        t = np.zeros((6, 3)) if traction is None else np.ascontiguousarray(traction, dtype=np.float64)
        assert t.shape == (6, 3), "traction: one 3-vector per macro face 2 d + side"
        return b, np.ascontiguousarray(t)

    def load_table_build(self):
        check(lib().igamt_load_table_build(self._h, _stream()))

    def load_table_get(self):
        torch = _torch()
        out = torch.empty((self.n_tile_ctrl, self.n_cols // 9, 7), dtype=torch.float64, device="cuda")
        check(lib().igamt_load_table_get(self._h, _ptr(out), _stream()))
        return out

    def load_workspace(self):
        nb = C.c_int64()
        check(lib().igamt_load_workspace_bytes(self._h, C.byref(nb)))
        return self._empty_bytes(nb.value)

    def load_fit(self, body, traction=None, out=None):
        """Projection coefficients [n_tiles, 7, 3, n_pi] of the body force and the face tractions."""
        torch = _torch()
        b, t = self._loads(body, traction)
        if out is None:
            out = torch.empty((self.n_tiles, 7, 3, self.n_cols // 9), dtype=torch.float64, device="cuda")
        check(lib().igamt_load_fit(self._h, b.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p),
                                   _ptr(out), _stream()))
        return out

    def load_gather(self, coef, out=None):
        torch = _torch()
        out = torch.empty(self.n_dofs, dtype=torch.float64, device="cuda") if out is None else out
        check(lib().igamt_load_gather(self._h, _ptr(coef), _ptr(out), _stream()))
        return out

    def load_assemble(self, body, traction=None, out=None, workspace=None):
        """The global load vector f^pi [n_dofs] (eq. (53)) on the device."""
        torch = _torch()
        b, t = self._loads(body, traction)
        out = torch.empty(self.n_dofs, dtype=torch.float64, device="cuda") if out is None else out
        workspace = self.load_workspace() if workspace is None else workspace
        check(lib().igamt_load_assemble(self._h, b.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p),
                                        _ptr(out), _ptr(workspace), _stream()))
        return out

    def uf_grad(self, body, traction, u, workspace=None):
        """(u . f^pi, d(u . f^pi)/d macro control points) with u fixed; f^pi is the load vector of
        load_assemble for the same body force and tractions (needs load_table_build)."""
        torch = _torch()
        b, t = self._loads(body, traction)
        u = self._vec(u)
        grad = torch.empty(self.macro_ctrl_shape, dtype=torch.float64, device="cuda")
        val = torch.empty(1, dtype=torch.float64, device="cuda")
        if workspace is None:
            nb = C.c_int64()
            check(lib().igamt_uf_grad_workspace_bytes(self._h, C.byref(nb)))
            workspace = self._empty_bytes(nb.value)
        check(lib().igamt_uf_grad(self._h, b.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p), _ptr(u),
                                  _ptr(grad), _ptr(val), _ptr(workspace), _stream()))
        return val, grad

    # ---- matrix-free product K u (eq. (74)) -----------------------------------------------
    def linop_workspace(self, prec="f64", slab_tiles=0):
        nb = C.c_int64()
        check(lib().igamt_linop_workspace_bytes(self._h, _prec(prec), int(slab_tiles), C.byref(nb)))
        return self._empty_bytes(nb.value)

    def _vec(self, u):
        torch = _torch()
        assert u.is_cuda and u.dtype == torch.float64 and u.is_contiguous() and u.numel() == self.n_dofs
        return u

    def apply_blocks(self, blocks, u, prec="f64", out=None, workspace=None):
        """y = K u from the tile blocks of contract() (the global matrix is never formed)."""
        torch = _torch()
        u = self._vec(u)
        out = torch.empty(self.n_dofs, dtype=torch.float64, device="cuda") if out is None else out
        workspace = self.linop_workspace(prec) if workspace is None else workspace
        check(lib().igamt_apply_blocks(self._h, _prec(prec), _ptr(blocks), _ptr(u), _ptr(out), _ptr(workspace),
                                       _stream()))
        return out

    def linop(self, coef, u, prec="f64", slab_tiles=512, out=None, workspace=None):
        """y = K u on the fly from the table and the coefficients of fit(), slab by slab."""
        torch = _torch()
        u = self._vec(u)
        out = torch.empty(self.n_dofs, dtype=torch.float64, device="cuda") if out is None else out
        workspace = self.linop_workspace(prec, slab_tiles) if workspace is None else workspace
        check(lib().igamt_linop(self._h, _prec(prec), int(slab_tiles), _ptr(coef), _ptr(u), _ptr(out),
                                _ptr(workspace), _stream()))
        return out

    def face_mask(self, faces):
        """uint8 [n_dofs] on the device, 1 on the dofs of the control points on the given macro
        faces (2 d + side; side 0: xi_d = 0)."""
        torch = _torch()
        GX, GY, GZ = self.grid
        idx = np.indices((GZ, GY, GX))
        on = np.zeros(GX * GY * GZ, bool)
        for face in faces:
            d, side = divmod(int(face), 2)
            along = (idx[2], idx[1], idx[0])[d].reshape(-1)
            on |= along == ((GX, GY, GZ)[d] - 1 if side else 0)
        return torch.from_numpy(np.repeat(on, 3).astype(np.uint8)).cuda()

    def pcg(self, blocks, f, fixed, prec="f64", rtol=1e-10, max_iter=10000, u0=None, workspace=None):
        """Jacobi-preconditioned CG on K u = f with u = 0 on the dofs where fixed != 0, using the
        matrix-free product of the tile blocks; returns (u, iterations, relative residual)."""
        torch = _torch()
        f = self._vec(f)
        assert fixed.is_cuda and fixed.dtype == torch.uint8 and fixed.numel() == self.n_dofs
        u = torch.zeros_like(f) if u0 is None else self._vec(u0).clone()
        if workspace is None:
            nb = C.c_int64()
            check(lib().igamt_pcg_workspace_bytes(self._h, C.byref(nb)))
            workspace = self._empty_bytes(nb.value)
        it, res = C.c_int32(), C.c_double()
        check(lib().igamt_pcg(self._h, _prec(prec), _ptr(blocks), _ptr(f), _ptr(fixed), _ptr(u), float(rtol),
                              int(max_iter), _ptr(workspace), _stream(), C.byref(it), C.byref(res)))
        return u, it.value, res.value

    # ---- volume and its sensitivity (eq. (14)-(19), (25)-(26), (66)-(67)) ----------------
    def volume_table_build(self):
        check(lib().igamt_volume_table_build(self._h, _stream()))

    def volume_table_get(self):
        """(t^h, t_pi) as float64 [n_pi] device tensors."""
        torch = _torch()
        n = self.n_cols // 9
        t = torch.empty(n, dtype=torch.float64, device="cuda")
        tp = torch.empty(n, dtype=torch.float64, device="cuda")
        check(lib().igamt_volume_table_get(self._h, _ptr(t), _ptr(tp), _stream()))
        return t, tp

    def volume_workspace(self):
        nb = C.c_int64()
        check(lib().igamt_volume_workspace_bytes(self._h, C.byref(nb)))
        return self._empty_bytes(nb.value)

    def volume(self, grad=False, workspace=None):
        """(V [1], tile volumes [n_tiles], dV/dm [n_macro_ctrl, 3] or None) on the device."""
        torch = _torch()
        workspace = self.volume_workspace() if workspace is None else workspace
        v = torch.empty(1, dtype=torch.float64, device="cuda")
        tv = torch.empty(self.n_tiles, dtype=torch.float64, device="cuda")
        g = torch.empty((self.n_macro_ctrl, 3), dtype=torch.float64, device="cuda") if grad else None
        check(lib().igamt_volume(self._h, _ptr(tv), _ptr(v), _ptr(g) if grad else None, _ptr(workspace),
                                 _stream()))
        return v, tv, g

    def volume_noalloc(self, grad=False, v=None, tv=None, g=None):
        """volume() through igamt_volume_noalloc: the library's static device scratch replaces the
        workspace (no allocation inside the call; outputs may be passed in to allocate none here)."""
        torch = _torch()
        v = torch.empty(1, dtype=torch.float64, device="cuda") if v is None else v
        tv = torch.empty(self.n_tiles, dtype=torch.float64, device="cuda") if tv is None else tv
        if grad and g is None:
            g = torch.empty((self.n_macro_ctrl, 3), dtype=torch.float64, device="cuda")
        check(lib().igamt_volume_noalloc(self._h, _ptr(tv), _ptr(v), _ptr(g) if grad else None, _stream()))
        return v, tv, g if grad else None

    # ---- projection error and adaptive degree (eq. (59), (65)) -----------------------------
    def eproj(self, E, nu, q=None, n_sample=5, per_tile=False):
        """E_proj (eq. (59)) at degree q (an int or a triple; default the plan's); with per_tile, also
        the per-tile maxima."""
        torch = _torch()
        q = self.q_dir if q is None else q
        qd = np.ascontiguousarray(((int(q),) * 3 if np.ndim(q) == 0 else tuple(q)), dtype=np.int32)
        te = torch.empty(self.n_tiles, dtype=torch.float64, device="cuda") if per_tile else None
        e = C.c_double()
        check(lib().igamt_eproj_aniso(self._h, float(E), float(nu), qd.ctypes.data_as(C.c_void_p), int(n_sample),
                                      _ptr(te) if per_tile else None, C.byref(e), _stream()))
        return (e.value, te) if per_tile else e.value

    def select_q(self, E, nu, tol=1e-3, q_max=6, n_sample=5):
        """Eq. (65): (q, E_proj(q)) for the first q from the macro degree with E_proj <= tol, or
        (None, E_proj(q_max))."""
        q, e = C.c_int32(), C.c_double()
        check(lib().igamt_select_q(self._h, float(E), float(nu), float(tol), int(q_max), int(n_sample),
                                   C.byref(q), C.byref(e), _stream()))
        return (None if q.value < 0 else q.value), e.value

    def select_q_aniso(self, E, nu, tol=1e-3, q_max=6, n_sample=5):
        """Anisotropic degrees (q_x, q_y, q_z) by the per-direction raise rule, with their E_proj, or
        (None, E_proj) when every direction reached q_max."""
        q = np.zeros(3, dtype=np.int32)
        e = C.c_double()
        check(lib().igamt_select_q_aniso(self._h, float(E), float(nu), float(tol), int(q_max), int(n_sample),
                                         q.ctypes.data_as(C.c_void_p), C.byref(e), _stream()))
        return (None if q[0] < 0 else tuple(int(v) for v in q)), e.value

    # ---- batches of designs of the plan's tile family -------------------------------------
    def _batch_ctrl(self, ctrls):
        torch = _torch()
        assert ctrls.is_cuda and ctrls.dtype == torch.float64 and ctrls.is_contiguous()
        assert ctrls.numel() == ctrls.shape[0] * 3 * self.n_tile_ctrl
        return int(ctrls.shape[0])

    def tables_build_batch(self, ctrls, gate=None, out=None):
        """Exact tables of a batch of designs (device tile control points [B, n_tile_ctrl, 3]) into
        a dense [B, n_pairs, n_cols] tensor; with an int32 gate [B], only designs with gate != 0."""
        torch = _torch()
        B = self._batch_ctrl(ctrls)
        if out is None:
            out = torch.empty((B, self.n_pairs, self.n_cols), dtype=torch.float64, device="cuda")
        if gate is not None:
            assert gate.is_cuda and gate.dtype == torch.int32 and gate.numel() == B
        check(lib().igamt_tables_build_batch(self._h, _ptr(ctrls), B, None if gate is None else _ptr(gate),
                                             _ptr(out), _stream()))
        return out

    def tables_build_rows_batch(self, ctrls, rows):
        torch = _torch()
        B = self._batch_ctrl(ctrls)
        rows = rows.to(device="cuda", dtype=torch.int32).contiguous()
        out = torch.empty((B, rows.numel(), self.n_cols), dtype=torch.float64, device="cuda")
        check(lib().igamt_tables_build_rows_batch(self._h, _ptr(ctrls), B, _ptr(rows), int(rows.numel()), _ptr(out),
                                                  _stream()))
        return out

    def tables_from_pod_batch(self, mean, basis, coeffs, scale=1.0, out=None):
        torch = _torch()
        coeffs = coeffs.contiguous()
        B, r = int(coeffs.shape[0]), int(basis.shape[0])
        work = torch.empty(lib().igamt_pod_batch_work_doubles(r, B), dtype=torch.float64, device="cuda")
        if out is None:
            out = torch.empty((B, self.n_pairs, self.n_cols), dtype=torch.float64, device="cuda")
        check(lib().igamt_tables_from_pod_batch(self._h, _ptr(mean), _ptr(basis), r, _ptr(coeffs), B, float(scale),
                                                _ptr(work), _ptr(out), _stream()))
        return out

    def tables_rows_check_batch(self, tables, rows, exact_rows, tol):
        """Per-design (relative error on the rows [B], int32 gate [B]), left on the device."""
        torch = _torch()
        B = int(tables.shape[0])
        rows = rows.to(device="cuda", dtype=torch.int32).contiguous()
        err = torch.empty(B, dtype=torch.float64, device="cuda")
        gate = torch.empty(B, dtype=torch.int32, device="cuda")
        check(lib().igamt_tables_rows_check_batch(self._h, _ptr(tables.contiguous()), B, _ptr(rows),
                                                  int(rows.numel()), _ptr(exact_rows.contiguous()), float(tol),
                                                  _ptr(err), _ptr(gate), _stream()))
        return err, gate


def spmv(row_ptr, col_idx, values, x, out=None):
    torch = _torch()
    prec = F64 if values.dtype == torch.float64 else F32
    out = torch.empty_like(x) if out is None else out
    check(lib().igamt_spmv(prec, row_ptr.numel() - 1, _ptr(row_ptr), _ptr(col_idx), _ptr(values), _ptr(x),
                           _ptr(out), _stream()))
    return out
