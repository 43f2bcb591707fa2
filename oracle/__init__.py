"""CPU oracle for SM-compressed integer matrices (arXiv 1303.0270, Method 1).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It wraps the plain C
implementation in ``ccmref.c`` (bit-at-a-time reader and writer, exact
``__int128`` arithmetic) through ctypes and shares no code with the GPU
library.

Every matrix-valued operation follows the definition "decode -> exact integer
arithmetic -> encode at the minimal width of the result" (see ``ccmref.h`` for
the readings taken where the paper is silent and for the parity pins).

The module-level functions use the library built from ``ccmref.c``;
``Oracle(path)`` binds the same API to another build of that source (the
mutation tests use it to show that the pins catch planted mistakes).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from ._build import build_oracle, library_path

OK, E_INVAL, E_SHAPE, E_RANGE, E_OVERFLOW = 0, -1, -2, -3, -4
_NAMES = {E_INVAL: "invalid argument", E_SHAPE: "shape mismatch", E_RANGE: "out of range",
          E_OVERFLOW: "overflow"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle: {_NAMES.get(code, code)}")
        self.code = code


class _Matrix(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("vmin", ctypes.c_int64), ("vmax", ctypes.c_int64),
                ("bits", ctypes.c_int32), ("is_signed", ctypes.c_int32),
                ("words", ctypes.c_uint64), ("payload", ctypes.c_void_p)]


class _Vlb(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("vmin", ctypes.c_int64), ("vmax", ctypes.c_int64),
                ("k", ctypes.c_int32), ("is_signed", ctypes.c_int32),
                ("nbits", ctypes.c_uint64), ("words", ctypes.c_uint64),
                ("payload", ctypes.c_void_p)]


_I64P = ctypes.POINTER(ctypes.c_int64)
_U64P = ctypes.POINTER(ctypes.c_uint64)
_MP = ctypes.POINTER(_Matrix)
_VP = ctypes.POINTER(_Vlb)
_SIGNATURES = {
    "ccmref_bitlen": (ctypes.c_int, [ctypes.c_uint64]),
    "ccmref_sm_width": (ctypes.c_int, [ctypes.c_uint64]),
    "ccmref_width": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]),
    "ccmref_words": (ctypes.c_uint64, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]),
    "ccmref_plan": (ctypes.c_int, [_I64P, ctypes.c_int64, ctypes.c_int64, _MP]),
    "ccmref_compress": (ctypes.c_int, [_I64P, _MP]),
    "ccmref_decompress": (ctypes.c_int, [_MP, _I64P]),
    "ccmref_get": (ctypes.c_int, [_MP, ctypes.c_int64, ctypes.c_int64, _I64P]),
    "ccmref_encode_run": (None, [_I64P, ctypes.c_int64, ctypes.c_int32, _U64P]),
    "ccmref_decode_run": (None, [_U64P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _I64P]),
    "ccmref_header": (None, [_MP, ctypes.POINTER(ctypes.c_uint8)]),
    "ccmref_add_dense": (ctypes.c_int, [_MP, _MP, _I64P]),
    "ccmref_scale_dense": (ctypes.c_int, [_MP, ctypes.c_int64, _I64P]),
    "ccmref_matvec_rows": (ctypes.c_int, [_MP, _I64P, ctypes.c_int64, ctypes.c_int64, _I64P]),
    "ccmref_matmul_check": (ctypes.c_int, [_MP, _MP]),
    "ccmref_matmul_dense": (ctypes.c_int, [_MP, _MP, _I64P]),
    "ccmref_matmul_entries": (ctypes.c_int, [_MP, _MP, _I64P, _I64P, ctypes.c_int64, _I64P]),
    "ccmref_compress_cm": (ctypes.c_int, [_I64P, _MP]),
    "ccmref_decompress_cm": (ctypes.c_int, [_MP, _I64P]),
    "ccmref_get_cm": (ctypes.c_int, [_MP, ctypes.c_int64, ctypes.c_int64, _I64P]),
    "ccmref_matvec_cm": (ctypes.c_int, [_MP, _I64P, _I64P]),
    "ccmref_matvec_t": (ctypes.c_int, [_MP, _I64P, _I64P]),
    "ccmref_matvec_t_cm": (ctypes.c_int, [_MP, _I64P, _I64P]),
    "ccmref_header_cm": (None, [_MP, ctypes.POINTER(ctypes.c_uint8)]),
    "ccmref_method_info_of": (ctypes.c_int, [_I64P, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_void_p]),
    "ccmref_eta2_model": (ctypes.c_double, [ctypes.POINTER(ctypes.c_double), ctypes.c_int32]),
    "ccmref_vlb_width": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32]),
    "ccmref_vlb_plan": (ctypes.c_int, [_I64P, ctypes.c_int64, ctypes.c_int64, _VP]),
    "ccmref_vlb_compress": (ctypes.c_int, [_I64P, _VP]),
    "ccmref_vlb_decompress": (ctypes.c_int, [_VP, _I64P]),
    "ccmref_vlb_get": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, _I64P]),
    "ccmref_vlb_matvec": (ctypes.c_int, [_VP, _I64P, _I64P]),
    "ccmref_vlb_offsets": (ctypes.c_int, [_VP, ctypes.c_int64, _U64P]),
    "ccmref_frac_bits": (ctypes.c_int, [ctypes.c_double, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]),
    "ccmref_quantize_f64": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                                           ctypes.c_int32, _I64P]),
    "ccmref_quantize_f32": (ctypes.c_int, [ctypes.POINTER(ctypes.c_float), ctypes.c_int64,
                                           ctypes.c_int32, _I64P]),
    "ccmref_dequantize_f64": (None, [_I64P, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_double)]),
    "ccmref_dequantize_f32": (None, [_I64P, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_float)]),
    "ccmref_header_fx": (None, [_MP, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8)]),
}


def _i64(a: np.ndarray):
    return a.ctypes.data_as(_I64P)


def _u64(a: np.ndarray):
    return a.ctypes.data_as(_U64P)


def _check(rc: int) -> None:
    if rc != OK:
        raise OracleError(rc)


@dataclass
class Packed:
    """The oracle's compressed matrix: header fields plus host payload words."""
    rows: int
    cols: int
    vmin: int
    vmax: int
    bits: int
    is_signed: bool
    payload: np.ndarray  # uint64 bitstrings, floor(rows*cols*bits/64)+1 of them

    @property
    def words(self) -> int:
        return int(self.payload.size)

    def _struct(self) -> _Matrix:
        return _Matrix(self.rows, self.cols, self.vmin, self.vmax, self.bits,
                       1 if self.is_signed else 0, self.words,
                       self.payload.ctypes.data_as(ctypes.c_void_p))

    def payload_bytes(self) -> bytes:
        return self.payload.astype("<u8").tobytes()


class _MethodInfo(ctypes.Structure):
    _fields_ = [("vmin", ctypes.c_int64), ("vmax", ctypes.c_int64),
                ("sm_bits", ctypes.c_int32), ("vlb_k", ctypes.c_int32),
                ("sm_nbits", ctypes.c_uint64), ("vlb_nbits", ctypes.c_uint64),
                ("eta1", ctypes.c_double), ("eta2", ctypes.c_double),
                ("method", ctypes.c_int32), ("pad", ctypes.c_int32)]


@dataclass
class VlbPacked:
    """The oracle's Method 2 (VLB) matrix: k-bit length fields, each followed by
    its element's own minimal width."""
    rows: int
    cols: int
    vmin: int
    vmax: int
    k: int
    is_signed: bool
    nbits: int
    payload: np.ndarray  # uint64 bitstrings, floor(nbits/64)+1 of them

    @property
    def words(self) -> int:
        return int(self.payload.size)

    def _struct(self) -> _Vlb:
        return _Vlb(self.rows, self.cols, self.vmin, self.vmax, self.k,
                    1 if self.is_signed else 0, self.nbits, self.words,
                    self.payload.ctypes.data_as(ctypes.c_void_p))


class Oracle:
    """The oracle's API bound to one build of ``ccmref.c``."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        self._lib = lib
        self.path = path

    # -- bit-length and width ------------------------------------------------
    def bitlen(self, u: int) -> int:
        return int(self._lib.ccmref_bitlen(u))

    def sm_width(self, sup: int) -> int:
        return int(self._lib.ccmref_sm_width(sup))

    def width(self, vmin: int, vmax: int) -> tuple[int, bool]:
        b, s = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.ccmref_width(vmin, vmax, ctypes.byref(b), ctypes.byref(s)))
        return int(b.value), bool(s.value)

    def words(self, rows: int, cols: int, bits: int) -> int:
        return int(self._lib.ccmref_words(rows, cols, bits))

    def packed_bytes(self, rows: int, cols: int, bits: int) -> int:
        """Closed-form compressed size: 64-byte header plus the bitstrings."""
        return 64 + 8 * self.words(rows, cols, bits)

    # -- compress / decompress / get ----------------------------------------
    def compress(self, dense) -> Packed:
        d = np.ascontiguousarray(np.asarray(dense, dtype=np.int64))
        if d.ndim != 2:
            raise OracleError(E_INVAL)
        m = _Matrix()
        _check(self._lib.ccmref_plan(_i64(d), d.shape[0], d.shape[1], ctypes.byref(m)))
        payload = np.zeros(int(m.words), dtype=np.uint64)
        m.payload = payload.ctypes.data_as(ctypes.c_void_p)
        _check(self._lib.ccmref_compress(_i64(d), ctypes.byref(m)))
        return Packed(int(m.rows), int(m.cols), int(m.vmin), int(m.vmax), int(m.bits),
                      bool(m.is_signed), payload)

    def decompress(self, p: Packed) -> np.ndarray:
        out = np.empty((p.rows, p.cols), dtype=np.int64)
        m = p._struct()
        _check(self._lib.ccmref_decompress(ctypes.byref(m), _i64(out)))
        return out

    def get(self, p: Packed, i: int, j: int) -> int:
        v = ctypes.c_int64()
        m = p._struct()
        _check(self._lib.ccmref_get(ctypes.byref(m), i, j, ctypes.byref(v)))
        return int(v.value)

    def header(self, p: Packed) -> bytes:
        buf = (ctypes.c_uint8 * 64)()
        m = p._struct()
        self._lib.ccmref_header(ctypes.byref(m), buf)
        return bytes(buf)

    def header_of(self, rows: int, cols: int, vmin: int, vmax: int) -> bytes:
        """Header of the rows x cols matrix whose exact extremes are vmin and
        vmax (its width from the width rule, its bitstring count from the
        closed form); no payload is needed to form it."""
        bits, signed = self.width(vmin, vmax)
        m = _Matrix(rows, cols, vmin, vmax, bits, 1 if signed else 0,
                    self.words(rows, cols, bits), None)
        buf = (ctypes.c_uint8 * 64)()
        self._lib.ccmref_header(ctypes.byref(m), buf)
        return bytes(buf)

    def encode_run(self, vals, bits: int, nwords: int | None = None) -> np.ndarray:
        v = np.ascontiguousarray(np.asarray(vals, dtype=np.int64).ravel())
        n = v.size
        if nwords is None:
            nwords = (n * bits) // 64 + 1
        if nwords * 64 < n * bits:
            raise OracleError(E_INVAL)
        w = np.zeros(nwords, dtype=np.uint64)
        self._lib.ccmref_encode_run(_i64(v), n, bits, _u64(w))
        return w

    def decode_run(self, wds, n: int, bits: int, is_signed: bool) -> np.ndarray:
        w = np.ascontiguousarray(np.asarray(wds, dtype=np.uint64))
        if w.size * 64 < n * bits:
            raise OracleError(E_INVAL)
        out = np.empty(n, dtype=np.int64)
        self._lib.ccmref_decode_run(_u64(w), n, bits, 1 if is_signed else 0, _i64(out))
        return out

    # -- arithmetic -----------------------------------------------------------
    def add_dense(self, a: Packed, b: Packed) -> np.ndarray:
        out = np.empty((a.rows, a.cols), dtype=np.int64)
        ma, mb = a._struct(), b._struct()
        _check(self._lib.ccmref_add_dense(ctypes.byref(ma), ctypes.byref(mb), _i64(out)))
        return out

    def add(self, a: Packed, b: Packed) -> Packed:
        return self.compress(self.add_dense(a, b))

    def scale_dense(self, a: Packed, s: int) -> np.ndarray:
        out = np.empty((a.rows, a.cols), dtype=np.int64)
        ma = a._struct()
        _check(self._lib.ccmref_scale_dense(ctypes.byref(ma), s, _i64(out)))
        return out

    def scale(self, a: Packed, s: int) -> Packed:
        return self.compress(self.scale_dense(a, s))

    def matvec(self, a: Packed, x, row_begin: int = 0, row_end: int | None = None) -> np.ndarray:
        """y = A x modulo 2^64 for rows [row_begin, row_end)."""
        xv = np.ascontiguousarray(np.asarray(x, dtype=np.int64).ravel())
        if xv.size != a.cols:
            raise OracleError(E_SHAPE)
        if row_end is None:
            row_end = a.rows
        y = np.empty(max(row_end - row_begin, 0), dtype=np.int64)
        ma = a._struct()
        _check(self._lib.ccmref_matvec_rows(ctypes.byref(ma), _i64(xv), row_begin, row_end,
                                            _i64(y)))
        return y

    def matmul_check(self, a: Packed, b: Packed) -> None:
        ma, mb = a._struct(), b._struct()
        _check(self._lib.ccmref_matmul_check(ctypes.byref(ma), ctypes.byref(mb)))

    def matmul_dense(self, a: Packed, b: Packed) -> np.ndarray:
        out = np.empty((a.rows, b.cols), dtype=np.int64)
        ma, mb = a._struct(), b._struct()
        _check(self._lib.ccmref_matmul_dense(ctypes.byref(ma), ctypes.byref(mb), _i64(out)))
        return out

    def matmul(self, a: Packed, b: Packed) -> Packed:
        return self.compress(self.matmul_dense(a, b))

    def matmul_entries(self, a: Packed, b: Packed, ii, jj) -> np.ndarray:
        i = np.ascontiguousarray(np.asarray(ii, dtype=np.int64).ravel())
        j = np.ascontiguousarray(np.asarray(jj, dtype=np.int64).ravel())
        out = np.empty(i.size, dtype=np.int64)
        ma, mb = a._struct(), b._struct()
        _check(self._lib.ccmref_matmul_entries(ctypes.byref(ma), ctypes.byref(mb), _i64(i),
                                               _i64(j), i.size, _i64(out)))
        return out


    # -- column-major unravel ---------------------------------------------------
    # A column-major matrix is a Packed whose rows/cols are A's and whose
    # stream holds element (i, j) at index j*rows + i.
    def compress_cm(self, dense) -> Packed:
        d = np.ascontiguousarray(np.asarray(dense, dtype=np.int64))
        if d.ndim != 2:
            raise OracleError(E_INVAL)
        m = _Matrix()
        _check(self._lib.ccmref_plan(_i64(d), d.shape[0], d.shape[1], ctypes.byref(m)))
        payload = np.zeros(int(m.words), dtype=np.uint64)
        m.payload = payload.ctypes.data_as(ctypes.c_void_p)
        _check(self._lib.ccmref_compress_cm(_i64(d), ctypes.byref(m)))
        return Packed(int(m.rows), int(m.cols), int(m.vmin), int(m.vmax), int(m.bits),
                      bool(m.is_signed), payload)

    def decompress_cm(self, p: Packed) -> np.ndarray:
        out = np.empty((p.rows, p.cols), dtype=np.int64)
        m = p._struct()
        _check(self._lib.ccmref_decompress_cm(ctypes.byref(m), _i64(out)))
        return out

    def get_cm(self, p: Packed, i: int, j: int) -> int:
        v = ctypes.c_int64()
        m = p._struct()
        _check(self._lib.ccmref_get_cm(ctypes.byref(m), i, j, ctypes.byref(v)))
        return int(v.value)

    def _mv(self, fn, a: Packed, x, nin: int, nout: int) -> np.ndarray:
        xv = np.ascontiguousarray(np.asarray(x, dtype=np.int64).ravel())
        if xv.size != nin:
            raise OracleError(E_SHAPE)
        y = np.empty(nout, dtype=np.int64)
        ma = a._struct()
        _check(fn(ctypes.byref(ma), _i64(xv), _i64(y)))
        return y

    def matvec_cm(self, a: Packed, x) -> np.ndarray:
        """y = A x for a column-major A."""
        return self._mv(self._lib.ccmref_matvec_cm, a, x, a.cols, a.rows)

    def matvec_t(self, a: Packed, x) -> np.ndarray:
        """y = A^T x for a row-major A (x: rows values)."""
        return self._mv(self._lib.ccmref_matvec_t, a, x, a.rows, a.cols)

    def matvec_t_cm(self, a: Packed, x) -> np.ndarray:
        """y = A^T x for a column-major A."""
        return self._mv(self._lib.ccmref_matvec_t_cm, a, x, a.rows, a.cols)

    def header_cm(self, p: Packed) -> bytes:
        buf = (ctypes.c_uint8 * 64)()
        m = p._struct()
        self._lib.ccmref_header_cm(ctypes.byref(m), buf)
        return bytes(buf)

    # -- floats in fixed point (Conclusion) ---------------------------------------
    def frac_bits(self, absmax: float, sig_bits: int) -> int:
        """Fraction bits f that keep sig_bits significant bits of the largest
        magnitude: f = sig_bits - 1 - floor(log2 absmax) (0 for absmax 0)."""
        f = ctypes.c_int32()
        _check(self._lib.ccmref_frac_bits(float(absmax), sig_bits, ctypes.byref(f)))
        return int(f.value)

    def quantize(self, v, frac_bits: int) -> np.ndarray:
        """q = round-half-to-even(v * 2^f) as int64 (v float32 or float64)."""
        a = np.asarray(v)
        q = np.empty(a.shape, dtype=np.int64)
        if a.dtype == np.float32:
            a = np.ascontiguousarray(a)
            _check(self._lib.ccmref_quantize_f32(a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                 a.size, frac_bits, _i64(q)))
        else:
            a = np.ascontiguousarray(a, dtype=np.float64)
            _check(self._lib.ccmref_quantize_f64(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 a.size, frac_bits, _i64(q)))
        return q

    def dequantize(self, q, frac_bits: int, dtype=np.float64) -> np.ndarray:
        """v = q * 2^-f: q to double (round half to even), scaled, and for
        float32 rounded once more."""
        qa = np.ascontiguousarray(np.asarray(q, dtype=np.int64))
        if np.dtype(dtype) == np.float32:
            v = np.empty(qa.shape, dtype=np.float32)
            self._lib.ccmref_dequantize_f32(_i64(qa), qa.size, frac_bits,
                                            v.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        else:
            v = np.empty(qa.shape, dtype=np.float64)
            self._lib.ccmref_dequantize_f64(_i64(qa), qa.size, frac_bits,
                                            v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return v

    def header_fx(self, p: Packed, frac_bits: int) -> bytes:
        buf = (ctypes.c_uint8 * 64)()
        m = p._struct()
        self._lib.ccmref_header_fx(ctypes.byref(m), frac_bits, buf)
        return bytes(buf)

    def header_fx_of(self, rows: int, cols: int, vmin: int, vmax: int, frac_bits: int) -> bytes:
        """Fixed-point header of the rows x cols matrix of quantized values
        with exact extremes vmin and vmax (no payload needed)."""
        bits, signed = self.width(vmin, vmax)
        m = _Matrix(rows, cols, vmin, vmax, bits, 1 if signed else 0,
                    self.words(rows, cols, bits), None)
        buf = (ctypes.c_uint8 * 64)()
        self._lib.ccmref_header_fx(ctypes.byref(m), frac_bits, buf)
        return bytes(buf)

    # -- choosing the method -----------------------------------------------------
    def method_info(self, dense) -> dict:
        """Both methods' bit counts and efficiencies (Eq. 15, 17) and the one
        using fewer bits (1 on a tie)."""
        d = np.ascontiguousarray(np.asarray(dense, dtype=np.int64))
        if d.ndim != 2:
            raise OracleError(E_INVAL)
        info = _MethodInfo()
        _check(self._lib.ccmref_method_info_of(_i64(d), d.shape[0], d.shape[1],
                                               ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in _MethodInfo._fields_ if f != "pad"}

    def eta2_model(self, pmf, k: int) -> float:
        """Eq. 29 for pmf[b-1] = P(bit-length b), b = 1..64, fixed k."""
        p = np.zeros(64, dtype=np.float64)
        q = np.asarray(pmf, dtype=np.float64).ravel()
        p[: q.size] = q
        return float(self._lib.ccmref_eta2_model(p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 k))

    # -- Method 2 (VLB) -------------------------------------------------------
    def vlb_width(self, v: int, is_signed: bool) -> int:
        return int(self._lib.ccmref_vlb_width(v, 1 if is_signed else 0))

    def vlb_compress(self, dense) -> VlbPacked:
        d = np.ascontiguousarray(np.asarray(dense, dtype=np.int64))
        if d.ndim != 2:
            raise OracleError(E_INVAL)
        m = _Vlb()
        _check(self._lib.ccmref_vlb_plan(_i64(d), d.shape[0], d.shape[1], ctypes.byref(m)))
        payload = np.zeros(int(m.words), dtype=np.uint64)
        m.payload = payload.ctypes.data_as(ctypes.c_void_p)
        _check(self._lib.ccmref_vlb_compress(_i64(d), ctypes.byref(m)))
        return VlbPacked(int(m.rows), int(m.cols), int(m.vmin), int(m.vmax), int(m.k),
                         bool(m.is_signed), int(m.nbits), payload)

    def vlb_decompress(self, p: VlbPacked) -> np.ndarray:
        m = p._struct()
        out = np.empty((p.rows, p.cols), dtype=np.int64)
        _check(self._lib.ccmref_vlb_decompress(ctypes.byref(m), _i64(out)))
        return out

    def vlb_get(self, p: VlbPacked, i: int, j: int) -> int:
        m = p._struct()
        v = ctypes.c_int64()
        _check(self._lib.ccmref_vlb_get(ctypes.byref(m), i, j, ctypes.byref(v)))
        return int(v.value)

    def vlb_offsets(self, p: VlbPacked, group: int = 32) -> np.ndarray:
        """Start bit of every element (i, j) with j % group == 0, as a
        rows x ceil(cols/group) array."""
        m = p._struct()
        ng = (p.cols + group - 1) // group
        out = np.empty((p.rows, ng), dtype=np.uint64)
        _check(self._lib.ccmref_vlb_offsets(ctypes.byref(m), group,
                                            out.ctypes.data_as(_U64P)))
        return out

    def vlb_matvec(self, p: VlbPacked, x) -> np.ndarray:
        m = p._struct()
        xv = np.ascontiguousarray(np.asarray(x, dtype=np.int64))
        if xv.size != p.cols:
            raise OracleError(E_SHAPE)
        y = np.empty(p.rows, dtype=np.int64)
        _check(self._lib.ccmref_vlb_matvec(ctypes.byref(m), _i64(xv), _i64(y)))
        return y


def _default() -> Oracle:
    path = library_path()
    if not os.path.exists(path):
        build_oracle()
    return Oracle(path)


_ORACLE = _default()

bitlen = _ORACLE.bitlen
sm_width = _ORACLE.sm_width
width = _ORACLE.width
words = _ORACLE.words
packed_bytes = _ORACLE.packed_bytes
compress = _ORACLE.compress
decompress = _ORACLE.decompress
get = _ORACLE.get
header = _ORACLE.header
header_of = _ORACLE.header_of
encode_run = _ORACLE.encode_run
decode_run = _ORACLE.decode_run
add_dense = _ORACLE.add_dense
add = _ORACLE.add
scale_dense = _ORACLE.scale_dense
scale = _ORACLE.scale
matvec = _ORACLE.matvec
matmul_check = _ORACLE.matmul_check
matmul_dense = _ORACLE.matmul_dense
matmul = _ORACLE.matmul
matmul_entries = _ORACLE.matmul_entries
compress_cm = _ORACLE.compress_cm
decompress_cm = _ORACLE.decompress_cm
get_cm = _ORACLE.get_cm
matvec_cm = _ORACLE.matvec_cm
matvec_t = _ORACLE.matvec_t
matvec_t_cm = _ORACLE.matvec_t_cm
header_cm = _ORACLE.header_cm
method_info = _ORACLE.method_info
eta2_model = _ORACLE.eta2_model
vlb_width = _ORACLE.vlb_width
vlb_compress = _ORACLE.vlb_compress
vlb_decompress = _ORACLE.vlb_decompress
vlb_get = _ORACLE.vlb_get
vlb_matvec = _ORACLE.vlb_matvec
vlb_offsets = _ORACLE.vlb_offsets
frac_bits = _ORACLE.frac_bits
quantize = _ORACLE.quantize
dequantize = _ORACLE.dequantize
header_fx = _ORACLE.header_fx
header_fx_of = _ORACLE.header_fx_of


def threads() -> int:
    """OpenMP threads the oracle's row loops use (OMP_NUM_THREADS or all cores)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    return len(os.sched_getaffinity(0))
