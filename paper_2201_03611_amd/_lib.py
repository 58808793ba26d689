"""ctypes declarations of librise.so (the C ABI in include/rise.h).

The library is loaded from this package directory.  There is no fallback: if
librise.so is missing or fails to load, importing the package raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librise.so")

RISE_OK = 0
STATUS_NAMES = {0: "RISE_OK", 1: "RISE_ERR_NULL", 2: "RISE_ERR_SHAPE", 3: "RISE_ERR_ALIAS",
                4: "RISE_ERR_DTYPE", 5: "RISE_ERR_UNSUPPORTED", 6: "RISE_ERR_WORKSPACE",
                7: "RISE_ERR_HIP"}

RISE_F32, RISE_BF16 = 0, 1
RISE_MODE_F32, RISE_MODE_BF16, RISE_MODE_BF16X3, RISE_MODE_BF16X6, RISE_MODE_FP8 = 0, 1, 2, 3, 4
RISE_OP_N, RISE_OP_T = 0, 1
RISE_PAD_CLAMP, RISE_PAD_ZERO = 0, 1


RISE_STENCIL_LDS_TILE, RISE_STENCIL_STREAM, RISE_STENCIL_LDS_PIPE, RISE_STENCIL_ASYNC = 0, 1, 2, 3


class RiseTile(ctypes.Structure):
    _fields_ = [("bm", ctypes.c_int32), ("bn", ctypes.c_int32), ("bk", ctypes.c_int32)]


class RiseStencilSchedule(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("rows", ctypes.c_int32)]


class RiseGemmProblem(ctypes.Structure):
    _fields_ = [("C", ctypes.c_void_p), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64), ("ldc", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("opB", ctypes.c_int32)]


class RiseStencilProblem(ctypes.Structure):
    _fields_ = [("out", ctypes.c_void_p), ("inp", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("H", ctypes.c_int64), ("W", ctypes.c_int64), ("ld_in", ctypes.c_int64),
                ("ld_out", ctypes.c_int64), ("k", ctypes.c_int32), ("pad", ctypes.c_int32)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SZ = ctypes.c_size_t
_INT = ctypes.c_int

# name -> (restype, argtypes)
SIGNATURES = {
    "rise_gemv_workspace": (_SZ, [_I64, _I64, _INT]),
    "rise_gemv_parts": (_I32, [_I64, _I64, _INT]),
    "rise_gemv": (_INT, [_P, _P, _I64, _INT, _P, _I64, _I64, _P, _SZ, _P]),
    "rise_gemv_noalloc": (_INT, [_P, _P, _I64, _INT, _P, _I64, _I64, _P]),
    "rise_stencil2d_iterate_max_fuse": (_INT, []),
    "rise_stencil2d_iterate_default_fuse": (_I32, [_I32, _I32]),
    "rise_stencil2d_iterate_workspace": (_SZ, [_I64, _I64, _INT, _INT, _I64, _INT]),
    "rise_stencil2d_iterate": (_INT, [_P, _I64, _P, _I64, _I64, _I64, _P, _INT, _INT, _INT, _I64,
                                      _INT, _P, _SZ, _P]),
    "rise_iterate_sum_workspace": (_SZ, [_I64, _I64, _I64]),
    "rise_iterate_sum_passes": (_I32, [_I64, _I64, _I64, ctypes.POINTER(_I32), _I32]),
    "rise_iterate_sum": (_INT, [_P, _P, _I64, _I64, _I64, _P, _SZ, _P]),
    "rise_status_string": (ctypes.c_char_p, [_INT]),
    "rise_last_error": (ctypes.c_char_p, []),
    "rise_gemm_tiles": (_I32, [_INT, ctypes.POINTER(RiseTile), _I32]),
    "rise_gemm_default_tile": (_INT, [_I64, _I64, _I64, _INT, ctypes.POINTER(RiseTile)]),
    "rise_gemm_workspace": (_SZ, [_I64, _I64, _I64, _INT, ctypes.POINTER(RiseTile)]),
    "rise_gemm": (_INT, [_P, _I64, _P, _INT, _I64, _INT, _P, _INT, _I64, _INT, _I64, _I64, _I64,
                         _INT, ctypes.POINTER(RiseTile), _P, _SZ, _P]),
    "rise_gemm_backward_workspace": (_SZ, [_I64, _I64, _I64, _INT]),
    "rise_gemm_backward": (_INT, [_P, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _I64, _I64, _I64,
                                  _I64, _INT, _P, _SZ, _P]),
    "rise_prep_bytes": (_SZ, [_I64, _I64, _INT]),
    "rise_prep_operand": (_INT, [_P, _I64, _I64, _P, _I64, _I64, _I64, _I64, _INT, _P]),
    "rise_stencil_schedules": (_I32, [ctypes.POINTER(RiseStencilSchedule), _I32]),
    "rise_stencil2d_default_schedule": (_INT, [_I64, _I64, _I32, _I32,
                                                ctypes.POINTER(RiseStencilSchedule)]),
    "rise_stencil2d": (_INT, [_P, _I64, _P, _I64, _I64, _I64, _P, _I32, _I32, _INT,
                              ctypes.POINTER(RiseStencilSchedule), _P]),
    "rise_conv2d_workspace": (_SZ, [_I32, _I32]),
    "rise_conv2d": (_INT, [_P, _P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _INT, _P, _SZ,
                           _P]),
    "rise_conv2d_backward_workspace": (_SZ, [_I32, _I32, _I32, _I32, _I32]),
    "rise_conv2d_backward": (_INT, [_P, _P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _I32,
                                    _INT, _P, _SZ, _P]),
    "rise_plan_create": (_INT, [ctypes.POINTER(_P), ctypes.POINTER(RiseGemmProblem), _I32,
                                ctypes.POINTER(RiseStencilProblem), _I32, ctypes.c_char_p, _P]),
    "rise_plan_launch": (_INT, [_P, _P]),
    "rise_plan_launch_direct": (_INT, [_P, _P]),
    "rise_plan_destroy": (_INT, [_P]),
    "rise_plan_items": (_I32, [_P]),
    "rise_plan_tile": (_INT, [_P, _I32, ctypes.POINTER(RiseTile)]),
    "rise_gemm_batched": (_INT, [ctypes.POINTER(RiseGemmProblem), _I32, _P]),
    "rise_stencil2d_batched": (_INT, [ctypes.POINTER(RiseStencilProblem), _I32, _P]),
    "rise_autotune_batched": (_INT, [ctypes.c_char_p, _P]),
    "rise_autotune_gemm": (_INT, [ctypes.c_char_p, _I64, _I64, _I64, _INT, _P]),
    "rise_autotune_stencil": (_INT, [ctypes.c_char_p, _I64, _I64, _I32, _P]),
    "rise_set_tune_cache": (_INT, [ctypes.c_char_p]),
    "rise_ceiling_copy": (_INT, [_P, _P, _SZ, _P]),
    "rise_ceiling_mfma_sink_floats": (_SZ, []),
    "rise_ceiling_mfma": (_INT, [_INT, _I64, _P, _SZ, ctypes.POINTER(ctypes.c_double), _P]),
    "rise_stencil2d_backward_workspace": (_SZ, [_I64, _I64, _I32, _I32]),
    "rise_stencil2d_backward": (_INT, [_P, _I64, _P, _P, _I64, _P, _I64, _I64, _I64, _P, _I32,
                                       _I32, _INT, _P, _SZ, _P]),
}


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python paper_2201_03611_amd/build.py` "
                          "(or __graft_entry__.build()) first; there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def exported_names():
    return list(SIGNATURES)
