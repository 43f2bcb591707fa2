"""ctypes binding of libccm.so (the C ABI declared in include/ccm.h).

Argument marshalling only: every step of every operation runs in the HIP
kernels of libccm.  Loading fails loudly when the library is missing; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libccm.so")

OK, E_INVAL, E_SHAPE, E_RANGE, E_OVERFLOW, E_NOMEM, E_DEVICE, E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
I32, I64 = 0, 1


class CcmError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = lib.ccm_status_str(status).decode() if lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")
        self.status = status


class Desc(ctypes.Structure):
    """Mirror of ccm_desc."""
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("vmin", ctypes.c_int64), ("vmax", ctypes.c_int64),
                ("bits", ctypes.c_int32), ("is_signed", ctypes.c_int32),
                ("words", ctypes.c_uint64), ("payload", ctypes.c_void_p)]


class Result(ctypes.Structure):
    """Mirror of ccm_result (64 bytes)."""
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("vmin", ctypes.c_int64), ("vmax", ctypes.c_int64),
                ("bits", ctypes.c_int32), ("is_signed", ctypes.c_int32),
                ("words", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("reserved1", ctypes.c_uint64)]


class VlbDesc(ctypes.Structure):
    """Mirror of ccm_vlb_desc."""
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("vmin", ctypes.c_int64), ("vmax", ctypes.c_int64),
                ("k", ctypes.c_int32), ("is_signed", ctypes.c_int32),
                ("nbits", ctypes.c_uint64), ("words", ctypes.c_uint64),
                ("gmax", ctypes.c_uint64),
                ("payload", ctypes.c_void_p), ("index", ctypes.c_void_p)]


class MethodInfo(ctypes.Structure):
    """Mirror of ccm_method_info."""
    _fields_ = [("vmin", ctypes.c_int64), ("vmax", ctypes.c_int64),
                ("sm_bits", ctypes.c_int32), ("vlb_k", ctypes.c_int32),
                ("sm_nbits", ctypes.c_uint64), ("vlb_nbits", ctypes.c_uint64),
                ("eta1", ctypes.c_double), ("eta2", ctypes.c_double),
                ("method", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int32
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(Desc)
_vdp = ctypes.POINTER(VlbDesc)

SIGNATURES = {
    "ccm_version": (ctypes.c_int, []),
    "ccm_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "ccm_words": (_u64, [_i64, _i64, _i32]),
    "ccm_packed_bytes": (_u64, [_i64, _i64, _i32]),
    "ccm_payload_capacity": (_u64, [_i64, _i64, _i32]),
    "ccm_width": (ctypes.c_int, [_i64, _i64, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "ccm_header_encode": (ctypes.c_int, [_dp, ctypes.POINTER(ctypes.c_uint8)]),
    "ccm_header_decode": (ctypes.c_int, [ctypes.POINTER(ctypes.c_uint8), _dp]),
    "ccm_range": (ctypes.c_int, [_vp, _i32, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                 _vp]),
    "ccm_compress_plan": (ctypes.c_int, [_vp, _i32, _i64, _i64, _dp, _vp]),
    "ccm_compress": (ctypes.c_int, [_vp, _i32, _dp, _vp]),
    "ccm_decompress": (ctypes.c_int, [_dp, _vp, _vp]),
    "ccm_get": (ctypes.c_int, [_dp, _i64, _i64, ctypes.POINTER(_i64), _vp]),
    "ccm_gather": (ctypes.c_int, [_dp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "ccm_add_plan": (ctypes.c_int, [_dp, _dp, _dp, _vp]),
    "ccm_add": (ctypes.c_int, [_dp, _dp, _dp, _vp]),
    "ccm_add_capacity": (_u64, [_dp, _dp]),
    "ccm_add_onepass": (ctypes.c_int, [_dp, _dp, _dp, _vp]),
    "ccm_scale_plan": (ctypes.c_int, [_dp, _i64, _dp]),
    "ccm_scale": (ctypes.c_int, [_dp, _i64, _dp, _vp]),
    "ccm_matvec": (ctypes.c_int, [_dp, _vp, _i32, _vp, _vp]),
    "ccm_matmul_scratch_bytes": (_u64, [_dp, _dp]),
    "ccm_matmul_plan": (ctypes.c_int, [_dp, _dp, _dp, _vp, _u64, _vp]),
    "ccm_matmul": (ctypes.c_int, [_dp, _dp, _dp, _vp, _u64, _vp]),
    "ccm_async_ws_bytes": (_u64, []),
    "ccm_add_async": (ctypes.c_int, [_dp, _dp, _vp, _u64, _vp, _vp]),
    "ccm_matmul_capacity": (_u64, [_dp, _dp]),
    "ccm_matmul_async": (ctypes.c_int, [_dp, _dp, _vp, _u64, _vp, _u64, _vp, _vp]),
    "ccm_result_desc": (ctypes.c_int, [ctypes.POINTER(Result), _vp, _dp]),
    "ccm_batch_create": (ctypes.c_int, [_dp, _i32, _i32, ctypes.c_char_p,
                                        ctypes.POINTER(_vp)]),
    "ccm_batch_set_io": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
    "ccm_batch_matvec": (ctypes.c_int, [_vp, _i32, _vp]),
    "ccm_batch_info": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_u64),
                                      ctypes.POINTER(_i32)]),
    "ccm_batch_destroy": (ctypes.c_int, [_vp]),
    "ccm_batch_ws_create": (ctypes.c_int, [_i32, _i64, _i32, ctypes.c_char_p,
                                           ctypes.POINTER(_vp)]),
    "ccm_batch_ws_destroy": (ctypes.c_int, [_vp]),
    "ccm_batch_matvec_dyn": (ctypes.c_int, [_vp, _dp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                            _i32, _vp]),
    "ccm_fill_uniform": (ctypes.c_int, [_vp, _i32, _i64, _i64, _i64, _u64, _u64, _u64, _vp]),
    "ccm_generate_plan": (ctypes.c_int, [_i64, _i64, _i64, _i64, _u64, _u64, _dp, _vp]),
    "ccm_generate": (ctypes.c_int, [_dp, _i64, _i64, _u64, _u64, _vp]),
    "ccm_method_plan": (ctypes.c_int, [_vp, _i32, _i64, _i64, ctypes.POINTER(MethodInfo), _vp]),
    "ccm_matvec_t_scratch_bytes": (_u64, [_dp]),
    "ccm_matvec_t": (ctypes.c_int, [_dp, _vp, _i32, _vp, _vp, _u64, _vp]),
    "ccm_matvec_t_noalloc": (ctypes.c_int, [_dp, _vp, _i32, _vp, _vp]),
    "ccm_compress_cm": (ctypes.c_int, [_vp, _i32, _dp, _vp]),
    "ccm_header_encode_cm": (ctypes.c_int, [_dp, ctypes.POINTER(ctypes.c_uint8)]),
    "ccm_header_decode_cm": (ctypes.c_int, [ctypes.POINTER(ctypes.c_uint8), _dp]),
    "ccm_vlb_index_bytes": (_u64, [_i64, _i64]),
    "ccm_vlb_payload_capacity": (_u64, [_u64]),
    "ccm_vlb_compress_plan": (ctypes.c_int, [_vp, _i32, _i64, _i64, _vp, _vdp, _vp]),
    "ccm_vlb_compress": (ctypes.c_int, [_vp, _i32, _vdp, _vp]),
    "ccm_vlb_decompress": (ctypes.c_int, [_vdp, _vp, _vp]),
    "ccm_vlb_get": (ctypes.c_int, [_vdp, _i64, _i64, ctypes.POINTER(_i64), _vp]),
    "ccm_vlb_matvec": (ctypes.c_int, [_vdp, _vp, _i32, _vp, _vp]),
    "ccm_float_absmax": (ctypes.c_int, [_vp, _i32, _i64, ctypes.POINTER(ctypes.c_double), _vp]),
    "ccm_float_frac_bits": (ctypes.c_int, [ctypes.c_double, _i32, ctypes.POINTER(_i32)]),
    "ccm_quantize": (ctypes.c_int, [_vp, _i32, _i64, _i32, _vp, _i32, ctypes.POINTER(_i64),
                                    ctypes.POINTER(_i64), _vp]),
    "ccm_compress_fx": (ctypes.c_int, [_vp, _i32, _i32, _dp, _vp]),
    "ccm_dequantize": (ctypes.c_int, [_vp, _i64, _i32, _i32, _vp, _vp]),
    "ccm_header_encode_fx": (ctypes.c_int, [_dp, _i32, ctypes.POINTER(ctypes.c_uint8)]),
    "ccm_header_decode_fx": (ctypes.c_int, [ctypes.POINTER(ctypes.c_uint8), _dp,
                                            ctypes.POINTER(_i32)]),
}


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            f"libccm.so not found at {path}: build it first (python -m "
            f"paper_1303_0270_amd.build, or __graft_entry__.build()).  There is no CPU "
            f"fallback.")
    handle = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(handle, name)
        fn.restype = res
        fn.argtypes = args
    return handle


lib = None
lib = load()


def check(status: int, what: str = "") -> None:
    if status != OK:
        raise CcmError(status, what)
