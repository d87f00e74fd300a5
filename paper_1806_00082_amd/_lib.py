"""ctypes loader for libwigner.so (the C ABI declared in include/wigner.h).

The library is built in-tree by ``paper_1806_00082_amd.build``.  There is no fallback:
if the shared object is missing every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwigner.so")

WK_OK, WK_EINVAL, WK_ECAPACITY, WK_EHIP = 0, -1, -2, -3
WK_FP64, WK_BF16, WK_FP16, WK_BF16X3, WK_FP16X3, WK_FP32 = 0, 1, 2, 3, 4, 5
WK_FULL, WK_HALF = 0, 1
(ST_N, ST_PAIRS, ST_ABS_X, ST_ABS_M, ST_NEEDED, ST_KEPT, ST_REGEN, ST_MIXED,
 ST_OVERFLOW, ST_OVERFLOW_STEP, ST_CUM_STEPS, ST_CUM_N, ST_CUM_PAIRS, ST_CUM_ANNIH_IN,
 ST_CUM_KEPT, ST_CUM_REGEN) = range(16)
ST_COUNT = 16

PREC = {"fp64": WK_FP64, "bf16": WK_BF16, "fp16": WK_FP16, "bf16x3": WK_BF16X3,
        "fp16x3": WK_FP16X3}


class WkMesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("n_m", ctypes.c_int32), ("hbar", ctypes.c_double)]


class SpGeom(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("n_m", ctypes.c_int32), ("n_k", ctypes.c_int32), ("M_min", ctypes.c_int32),
                ("pos_f64", ctypes.c_int32), ("m_bytes", ctypes.c_int32),
                ("vdt", ctypes.c_double), ("seed", ctypes.c_uint64)]


class SpParticles(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("M", ctypes.c_void_p),
                ("My", ctypes.c_void_p), ("s", ctypes.c_void_p), ("capacity", ctypes.c_int64),
                ("d_n", ctypes.c_void_p)]


# name -> (restype, argtypes)
_P = ctypes.c_void_p
_i32, _i64, _f32, _f64, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_size_t
_MP, _GP, _PP = ctypes.POINTER(WkMesh), ctypes.POINTER(SpGeom), ctypes.POINTER(SpParticles)
SIGNATURES = {
    "wk_last_error": (ctypes.c_char_p, []),
    "wk_version": (ctypes.c_int, []),
    "wk_device_count": (ctypes.c_int, []),
    "wk_trace_enable": (ctypes.c_int, [_i32]),
    "wk_trace_disable": (ctypes.c_int, []),
    "wk_trace_read": (ctypes.c_int, [ctypes.c_char_p, _P, _P]),
    "wk_trace_names": (ctypes.c_int, [ctypes.c_char_p, _sz]),
    "wk_kernel_eval": (ctypes.c_int, [_MP, _P, _i32, _P, _i32, _i32, _i32, _P, _P]),
    "wk_prepare": (ctypes.c_int, [_MP, _P]),
    "wk_kernel_bwd_workspace": (_sz, [_MP, _i32, _i32, _i32]),
    "wk_kernel_bwd": (ctypes.c_int, [_MP, _P, _i32, _P, _i32, _i32, _i32, _P, _P, _sz, _P]),
    "wk_gamma_tables": (ctypes.c_int, [_MP, _P, _i32, _i32, _i32, _f64, _P, _P, _P, _P, _P]),
    "sp_workspace_size": (_sz, [_GP]),
    "sp_init": (ctypes.c_int, [_GP, _P, _PP, _P, _P, _sz, _P]),
    "sp_step": (ctypes.c_int, [_GP, _P, _P, _P, _P, _P, _i32, _PP, _PP, _P, _i32, _P, _i64, _P, _P, _sz, _P]),
    "wk_sampling_guide": (ctypes.c_int, [_P, _i32, _i32, _i32, _P, _P]),
    "wk_kernel_tables": (ctypes.c_int, [_MP, _P, _i32, _P, _i32, _i32, _f64, _P, _P, _P, _P, _P, _i32, _P]),
    "sp_annihilate": (ctypes.c_int, [_GP, _PP, _PP, _P, _i32, _P, _i64, _P, _P, _sz, _P]),
    "sp_pairs_scratch_size": (_sz, [_GP, _i64]),
    "sp_annihilate_pairs": (ctypes.c_int, [_GP, _PP, _PP, _P, _i32, _P, _P, _sz, _P, _sz, _P]),
    "sp_density": (ctypes.c_int, [_GP, _P, _f64, _P, _P]),
    "sp_cells_to_evaluate": (ctypes.c_int, [_GP, _P, _i32, _i32, _P, _P, _P, _P, _sz, _P]),
    "sp_assign_slots": (ctypes.c_int, [_P, _P, _i32, _i32, _P, _P]),
    "wk_surrogate_fwd_workspace": (_sz, [_MP, _i32]),
    "wk_surrogate_fwd": (ctypes.c_int, [_MP, _i32, _P, _P, _P, _P, _i32, _P, _i32, _i32, _P, _P, _sz, _P]),
    "wk_surrogate_fwd_static_max": (_sz, []),
    "wk_surrogate_fwd_static": (ctypes.c_int, [_MP, _i32, _P, _P, _P, _P, _i32, _P, _i32, _i32, _P, _P]),
    "wk_surrogate_fwd_2d": (ctypes.c_int, [_MP, _i32, _P, _P, _P, _P, _P, _i32, _P, _i32, _P, _P]),
    "wk_surrogate_tables_2d": (ctypes.c_int, [_MP, _i32, _P, _P, _P, _P, _P, _i32, _P, _i32, _f64, _P, _P,
                                              _P, _P, _P, _i32, _P]),
    "wk_surrogate_workspace": (_sz, [_MP, _i32, _i32, _i32]),
    "wk_surrogate_bwd": (ctypes.c_int, [_MP, _i32, _P, _P, _P, _P, _i32, _P, _i32, _P, _P, _P, _P,
                                        _P, _P, _sz, _P]),
    "wk_mse_grad": (ctypes.c_int, [_P, _P, _i64, _f64, _P, _P, _P, _sz, _P]),
    "wk_sgd_update": (ctypes.c_int, [_P, _P, _i32, _f32, _P]),
}

_lib = None


class WignerError(RuntimeError):
    pass


def lib() -> ctypes.CDLL:
    """Load libwigner.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise WignerError(f"{LIB_PATH} is missing: build it with paper_1806_00082_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int, what: str) -> int:
    if rc != WK_OK:
        msg = lib().wk_last_error().decode(errors="replace")
        raise WignerError(f"{what} failed ({rc}): {msg}")
    return rc


def trace_read(name: str):
    """(total ms, launches) of a traced kernel since wk_trace_enable."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    check(lib().wk_trace_read(name.encode(), ctypes.byref(ms), ctypes.byref(cnt)), "wk_trace_read")
    return ms.value, cnt.value


def trace_names():
    buf = ctypes.create_string_buffer(8192)
    check(lib().wk_trace_names(buf, len(buf)), "wk_trace_names")
    return [n for n in buf.value.decode().split("\n") if n]
