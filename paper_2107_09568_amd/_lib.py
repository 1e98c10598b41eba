"""ctypes declarations of the libigamt C ABI (include/igamt.h)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libigamt.so")

status = C.c_int32
vp = C.c_void_p
i32 = C.c_int32
i64 = C.c_int64
f32 = C.c_float
f64 = C.c_double
P_i32 = C.POINTER(C.c_int32)
P_i64 = C.POINTER(C.c_int64)
P_f64 = C.POINTER(C.c_double)


class Spline3D(C.Structure):
    _fields_ = [("degree", i32 * 3), ("n_ctrl", i32 * 3), ("knots", P_f64 * 3), ("ctrl", P_f64), ("weights", P_f64)]


class PlanDesc(C.Structure):
    _fields_ = [("tiles", i32 * 3), ("box_mode", i32), ("q", i32), ("n_fit", i32), ("n_gauss", i32),
                ("anisotropic", i32), ("q_dir", i32 * 3)]


class Sizes(C.Structure):
    _fields_ = [(n, i64) for n in ("n_tiles", "n_tiles_pad", "n_pairs", "n_cols", "n_cols_pad", "n_tile_ctrl",
                                   "n_macro_ctrl", "n_global_ctrl", "n_dofs", "nnz")]


class MlpDesc(C.Structure):
    _fields_ = [("n_layers", i32), ("widths", i32 * 9), ("batch", i32)]


SIGNATURES = {
    "igamt_last_error": (C.c_char_p, []),
    "igamt_plan_create": (status, [C.POINTER(Spline3D), C.POINTER(Spline3D), C.POINTER(PlanDesc), C.POINTER(vp)]),
    "igamt_plan_destroy": (None, [vp]),
    "igamt_plan_sizes": (status, [vp, C.POINTER(Sizes)]),
    "igamt_plan_pairs": (status, [vp, vp]),
    "igamt_plan_csr": (status, [vp, vp, vp]),
    "igamt_plan_csr_device": (status, [vp, vp, vp, vp]),
    "igamt_set_macro_ctrl": (status, [vp, vp, i32, vp]),
    "igamt_set_tile_ctrl": (status, [vp, vp]),
    "igamt_set_tile_ctrl_device": (status, [vp, vp, vp]),
    "igamt_tables_build": (status, [vp, vp]),
    "igamt_tables_build_gated": (status, [vp, vp, vp]),
    "igamt_tables_set": (status, [vp, vp, vp]),
    "igamt_tables_get": (status, [vp, vp, vp]),
    "igamt_tables_build_rows": (status, [vp, vp, i32, vp, vp]),
    "igamt_workspace_bytes": (status, [vp, i32, P_i64, P_i64]),
    "igamt_fit": (status, [vp, f64, f64, i32, vp, vp]),
    "igamt_contract": (status, [vp, i32, vp, vp, vp]),
    "igamt_contract_products": (status, [vp, i32, vp, vp, vp]),
    "igamt_scatter": (status, [vp, i32, vp, vp, vp]),
    "igamt_assemble": (status, [vp, f64, f64, i32, vp, vp, vp]),
    "igamt_check": (status, [vp, vp, P_i64]),
    "igamt_grad_workspace_bytes": (status, [vp, i32, P_i64]),
    "igamt_uKu_grad": (status, [vp, f64, f64, i32, vp, vp, vp, vp, vp]),
    "igamt_spmv": (status, [i32, i64, vp, vp, vp, vp, vp, vp]),
    "igamt_pod_build": (status, [vp, i32, i64, i32, vp, vp, vp, vp, vp, vp]),
    "igamt_table_from_pod": (status, [vp, vp, vp, i32, vp, f64, vp]),
    "igamt_table_rows_error": (status, [vp, vp, i32, vp, vp, vp]),
    "igamt_table_rows_check": (status, [vp, vp, i32, vp, f64, vp, vp, vp]),
    "igamt_table_learned": (status, [vp, C.POINTER(MlpDesc), vp, vp, vp, vp, vp, vp, f64, vp, i32, vp, f64, vp, vp,
                                     vp]),
    "igamt_load_table_build": (status, [vp, vp]),
    "igamt_load_table_get": (status, [vp, vp, vp]),
    "igamt_load_workspace_bytes": (status, [vp, P_i64]),
    "igamt_load_fit": (status, [vp, vp, vp, vp, vp]),
    "igamt_load_gather": (status, [vp, vp, vp, vp]),
    "igamt_load_assemble": (status, [vp, vp, vp, vp, vp, vp]),
    "igamt_uf_grad_workspace_bytes": (status, [vp, P_i64]),
    "igamt_uf_grad": (status, [vp, vp, vp, vp, vp, vp, vp, vp]),
    "igamt_linop_workspace_bytes": (status, [vp, i32, i64, P_i64]),
    "igamt_apply_blocks": (status, [vp, i32, vp, vp, vp, vp, vp]),
    "igamt_linop": (status, [vp, i32, i64, vp, vp, vp, vp, vp]),
    "igamt_pcg_workspace_bytes": (status, [vp, P_i64]),
    "igamt_volume_table_build": (status, [vp, vp]),
    "igamt_volume_table_get": (status, [vp, vp, vp, vp]),
    "igamt_volume_workspace_bytes": (status, [vp, P_i64]),
    "igamt_volume": (status, [vp, vp, vp, vp, vp, vp]),
    "igamt_volume_noalloc": (status, [vp, vp, vp, vp, vp]),
    "igamt_eproj": (status, [vp, f64, f64, i32, i32, vp, C.POINTER(f64), vp]),
    "igamt_select_q": (status, [vp, f64, f64, f64, i32, i32, C.POINTER(i32), C.POINTER(f64), vp]),
    "igamt_eproj_aniso": (status, [vp, f64, f64, vp, i32, vp, C.POINTER(f64), vp]),
    "igamt_select_q_aniso": (status, [vp, f64, f64, f64, i32, i32, vp, C.POINTER(f64), vp]),
    "igamt_pcg": (status, [vp, i32, vp, vp, vp, vp, f64, i32, vp, vp, C.POINTER(i32), C.POINTER(f64)]),
    "igamt_tables_build_batch": (status, [vp, vp, i32, vp, vp, vp]),
    "igamt_tables_build_rows_batch": (status, [vp, vp, i32, vp, i32, vp, vp]),
    "igamt_tables_from_pod_batch": (status, [vp, vp, vp, i32, vp, i32, f64, vp, vp, vp]),
    "igamt_pod_batch_work_doubles": (i64, [i32, i32]),
    "igamt_tables_rows_check_batch": (status, [vp, vp, i32, vp, i32, vp, f64, vp, vp, vp]),
    "igamt_tables_learned_batch": (status, [vp, C.POINTER(MlpDesc), vp, vp, vp, vp, vp, vp, f64, vp, vp, i32, vp,
                                            f64, vp, vp, vp, vp, vp]),
    "igamt_mlp_n_params": (i64, [C.POINTER(MlpDesc)]),
    "igamt_mlp_forward": (status, [C.POINTER(MlpDesc), vp, vp, vp, vp, vp]),
    "igamt_mse_loss": (status, [C.POINTER(MlpDesc), vp, vp, vp, vp, vp]),
    "igamt_mlp_backward": (status, [C.POINTER(MlpDesc), vp, vp, vp, vp, vp, vp, vp]),
    "igamt_adam_step": (status, [vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp]),
}

_lib = None


def lib():
    """Load libigamt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2107_09568_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class IgamtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"igamt error {code}: {msg}")
        self.code = code


def check(code):
    if code != 0:
        raise IgamtError(code, lib().igamt_last_error().decode())
