"""ctypes declarations for libdmg.so (the C ABI in include/dmg.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmg.so")

DMG_OK = 0
STATUS_NAMES = {0: "DMG_OK", 1: "DMG_ERR_INVALID_ARG", 2: "DMG_ERR_DIMS", 3: "DMG_ERR_WORKSPACE",
                4: "DMG_ERR_NOT_SPD", 5: "DMG_ERR_NONFINITE", 6: "DMG_ERR_NO_CONVERGENCE",
                7: "DMG_ERR_HIP", 8: "DMG_ERR_UNSUPPORTED"}
DMG_FP64, DMG_FP32_IR = 0, 1
DMG_MESH_HOST_SETUP, DMG_MESH_MATRIX_FREE = 1, 2


class DmgError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code
        self.message = message


class Options(C.Structure):
    _fields_ = [("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("pre_order", C.c_int32 * 4), ("post_order", C.c_int32 * 4),
                ("coarsest_n", C.c_int32), ("precision", C.c_int32),
                ("inner_cycles", C.c_int32), ("use_graph", C.c_int32),
                ("tile_rows", C.c_int32), ("strip_kernel", C.c_int32), ("smoother", C.c_int32),
                ("coarse_gemv", C.c_int32), ("reserved", C.c_int32 * 4)]


_p = C.c_void_p
_i32 = C.c_int32
_st = C.c_int

SIGNATURES = {
    "dmg_default_options": (None, [C.POINTER(Options)]),
    "dmg_last_error": (C.c_char_p, []),
    "dmg_version": (C.c_char_p, []),
    "dmg_assemble_stencil": (_st, [_p, _p, _i32, _i32, _p, _p]),
    "dmg_workspace_bytes": (_st, [_i32, _i32, C.POINTER(Options), C.POINTER(C.c_size_t)]),
    "dmg_setup": (_st, [_p, _i32, _i32, C.POINTER(Options), _p, C.c_size_t, _p, C.POINTER(_p)]),
    "dmg_destroy": (None, [_p]),
    "dmg_refresh": (_st, [_p, _p, _p]),
    "dmg_refresh_assembled": (_st, [_p, _p, _p, _p]),
    "dmg_sweep": (_st, [_p, _i32, _i32, _p, _p, _p]),
    "dmg_hier_level": (_st, [_p, _i32, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_p), C.POINTER(_p)]),
    "dmg_stats": (_st, [_p, C.POINTER(_i32), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "dmg_vcycle": (_st, [_p, _p, _p, _p]),
    "dmg_residual_norm": (_st, [_p, _p, _p, C.POINTER(C.c_double), _p]),
    "dmg_residual_norm_noalloc": (_st, [_p, _p, _p, _i32, _i32, _p, _p]),
    "dmg_autotune": (_st, [_p, _p, _p, _i32, _i32, _p]),
    "dmg_hier_config": (_st, [_p, _i32, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32)]),
    "dmg_hier_sweep_config": (_st, [_p, _i32, _i32, C.POINTER(_i32), C.POINTER(_i32)]),
    "dmg_hier_inner_cycles": (_st, [_p, C.POINTER(_i32)]),
    "dmg_solve": (_st, [_p, _p, _p, C.c_double, _i32, C.POINTER(_i32), C.POINTER(C.c_double),
                        C.POINTER(C.c_double), _p]),
    "dmg_grad_K": (_st, [_p, _p, _p, _i32, _i32, _p, _p]),
    "dmg_transfer_create_mesh": (_st, [_i32, _i32, _p, _p, _p, _p, _i32, _i32, _i32, _i32, _p, C.POINTER(_p)]),
    "dmg_transfer_workspace_bytes": (_st, [_i32, _i32, C.c_int64, C.POINTER(C.c_size_t)]),
    "dmg_transfer_create": (_st, [_i32, _i32, _p, _p, _p, _p, _p, _p, _p, C.c_size_t, _p, C.POINTER(_p)]),
    "dmg_transfer_info": (_st, [_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "dmg_transfer_memory": (_st, [_p, C.POINTER(C.c_size_t), C.POINTER(C.c_int64)]),
    "dmg_transfer_copy_C": (_st, [_p, _p, _p, _p]),
    "dmg_transfer_from_grid": (_st, [_p, _p, _p, _p]),
    "dmg_transfer_to_grid": (_st, [_p, _p, _p, _p]),
    "dmg_transfer_destroy": (None, [_p]),
    "dmg_twolevel_create": (_st, [_i32, _i32, _p, _p, _p, _p, _p, _p, _i32, _i32, _i32, _p, C.POINTER(_p)]),
    "dmg_twolevel_info": (_st, [_p, C.POINTER(_i32), C.POINTER(C.c_int64), _p]),
    "dmg_twolevel_cycle": (_st, [_p, _p, _p, _p]),
    "dmg_twolevel_solve": (_st, [_p, _p, _p, C.c_double, _i32, C.POINTER(_i32), C.POINTER(C.c_double), _p, _p]),
    "dmg_twolevel_set_scaling": (_st, [_p, C.c_double]),
    "dmg_twolevel_scaling": (_st, [_p, _p, _i32, C.POINTER(C.c_double), _p, C.POINTER(_i32), _p]),
    "dmg_twolevel_destroy": (None, [_p]),
    "dmg_batch_workspace_bytes": (_st, [_i32, _p, _p, C.POINTER(Options), C.POINTER(C.c_size_t)]),
    "dmg_batch_setup": (_st, [_i32, _p, _p, _p, C.POINTER(Options), _p, C.c_size_t, _p, C.POINTER(_p)]),
    "dmg_batch_solve": (_st, [_p, _p, _p, C.c_double, _i32, _p, _p, _p]),
    "dmg_batch_autotune": (_st, [_p, _p, _p, _i32, _i32, _p]),
    "dmg_batch_config": (_st, [_p, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32)]),
    "dmg_batch_instance_orders": (_st, [_p, _i32, C.POINTER(_i32), C.POINTER(_i32)]),
    "dmg_batch_destroy": (None, [_p]),
}

_lib = None


def load() -> C.CDLL:
    """Load the in-tree libdmg.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_08109_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != DMG_OK:
        msg = load().dmg_last_error().decode(errors="replace")
        raise DmgError(status, msg)


def default_options(**overrides) -> Options:
    o = Options()
    load().dmg_default_options(C.byref(o))
    for k, v in overrides.items():
        if k in ("pre_order", "post_order"):
            getattr(o, k)[:] = list(v)
        else:
            setattr(o, k, int(v))
    return o
