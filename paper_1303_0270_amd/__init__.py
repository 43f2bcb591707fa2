"""ccm: linear algebra on SM-compressed integer matrices on AMD MI355X.

Paper: Paixao & Codeco Coelho, "Computable Compressed Matrices" (arXiv
1303.0270), Method 1 (Supreme Minimum).  Python binding of libccm (C ABI in
include/ccm.h): these functions only marshal arguments; every step runs in the
library's HIP kernels.  PyTorch provides device memory and streams.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import (E_INVAL, E_NOMEM, E_OVERFLOW, E_RANGE, E_SHAPE, E_UNSUPPORTED, I32, I64,
                   OK, CcmError, Desc, MethodInfo, Result, VlbDesc, check, lib)

__all__ = ["CMatrix", "CcmError", "compress", "decompress", "get", "gather", "add", "scale",
           "matvec_launcher",
           "matvec", "matvec_t", "matmul", "matmul_plan", "matmul_pack", "fill_uniform", "generate", "from_serialized", "words",
           "Pending", "async_ws", "add_async", "matmul_async", "matmul_capacity",
           "packed_bytes", "payload_capacity", "width", "Batch", "DynBatch",
           "method_info", "compress_auto",
           "VlbMatrix", "vlb_compress", "vlb_decompress", "vlb_get", "vlb_matvec",
           "vlb_matvec_launcher", "float_absmax", "float_frac_bits", "quantize", "dequantize",
           "compress_float", "decompress_float", "matvec_float"]


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.int32:
        return I32
    if t.dtype == torch.int64:
        return I64
    raise TypeError(f"int32 or int64 tensor expected, got {t.dtype}")


F32, F64 = 2, 3  # float dtype codes of the C ABI


def _float_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"float32 or float64 tensor expected, got {t.dtype}")


def _device_tensor(t: torch.Tensor, what: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    return t.contiguous()


def words(rows: int, cols: int, bits: int) -> int:
    return int(lib.ccm_words(rows, cols, bits))


def packed_bytes(rows: int, cols: int, bits: int) -> int:
    return int(lib.ccm_packed_bytes(rows, cols, bits))


def payload_capacity(rows: int, cols: int, bits: int) -> int:
    return int(lib.ccm_payload_capacity(rows, cols, bits))


def width(vmin: int, vmax: int) -> tuple[int, bool]:
    b, s = ctypes.c_int32(), ctypes.c_int32()
    check(lib.ccm_width(vmin, vmax, ctypes.byref(b), ctypes.byref(s)), "ccm_width")
    return int(b.value), bool(s.value)


class CMatrix:
    """A compressed matrix: its descriptor plus the device payload it owns.

    order "C": unravelled by row, `desc` describes the matrix itself.
    order "F": unravelled by column; the stream is the row-major stream of the
    transpose, which `desc` describes (rows and cols swapped).  `T` flips the
    order and swaps the shape without touching the payload."""

    def __init__(self, desc: Desc, payload: torch.Tensor | None = None, device=None,
                 order: str = "C"):
        if order not in ("C", "F"):
            raise ValueError("order must be 'C' or 'F'")
        self.desc = desc
        self.order = order
        if payload is None:
            cap = int(lib.ccm_payload_capacity(desc.rows, desc.cols, desc.bits))
            payload = torch.empty(cap, dtype=torch.uint8, device=device or "cuda")
        self.payload = payload
        self.desc.payload = payload.data_ptr()
        # fixed-point matrices (floats, Conclusion): the values are q 2^-frac_bits
        self.frac_bits = None

    rows = property(lambda self: int(self.desc.rows if self.order == "C" else self.desc.cols))
    cols = property(lambda self: int(self.desc.cols if self.order == "C" else self.desc.rows))
    vmin = property(lambda self: int(self.desc.vmin))
    vmax = property(lambda self: int(self.desc.vmax))
    bits = property(lambda self: int(self.desc.bits))
    is_signed = property(lambda self: bool(self.desc.is_signed))
    words = property(lambda self: int(self.desc.words))

    @property
    def shape(self):
        return (self.rows, self.cols)

    @property
    def nbytes(self) -> int:
        """Serialized size: 64-byte header plus 8*W payload bytes."""
        return 64 + 8 * self.words

    @property
    def T(self) -> "CMatrix":
        """The transpose: the same payload read in the other order."""
        d = Desc()
        ctypes.pointer(d)[0] = self.desc
        t = CMatrix(d, self.payload, order="F" if self.order == "C" else "C")
        t.frac_bits = self.frac_bits
        return t

    def header(self) -> bytes:
        buf = (ctypes.c_uint8 * 64)()
        if self.frac_bits is not None:
            _row_major(self, "header of a fixed-point matrix")
            check(lib.ccm_header_encode_fx(ctypes.byref(self.desc), self.frac_bits, buf),
                  "ccm_header_encode_fx")
        elif self.order == "C":
            check(lib.ccm_header_encode(ctypes.byref(self.desc), buf), "ccm_header_encode")
        else:
            check(lib.ccm_header_encode_cm(ctypes.byref(self.desc), buf), "ccm_header_encode_cm")
        return bytes(buf)

    def payload_bytes(self) -> bytes:
        """The canonical payload (W little-endian 64-bit bitstrings) as bytes."""
        torch.cuda.current_stream().synchronize()
        return bytes(self.payload[: 8 * self.words].cpu().numpy().tobytes())

    def serialize(self) -> bytes:
        return self.header() + self.payload_bytes()

    def __repr__(self):
        fx = "" if self.frac_bits is None else f", frac_bits={self.frac_bits}"
        return (f"CMatrix({self.rows}x{self.cols}, order={self.order}, bits={self.bits}, "
                f"signed={self.is_signed}, range=[{self.vmin}, {self.vmax}]{fx})")


def _row_major(m: CMatrix, what: str) -> None:
    if m.order != "C":
        raise CcmError(E_UNSUPPORTED, f"{what}: column-major operand (use .T or re-compress)")


def from_serialized(blob: bytes, device="cuda") -> CMatrix:
    """Rebuild a compressed matrix from header + payload bytes."""
    if len(blob) < 64:
        raise CcmError(E_INVAL, "from_serialized")
    d = Desc()
    hdr = (ctypes.c_uint8 * 64).from_buffer_copy(blob[:64])
    order = "F" if blob[7] & 2 else "C"
    fx = None
    if blob[7] & 4:
        f = ctypes.c_int32()
        check(lib.ccm_header_decode_fx(hdr, ctypes.byref(d), ctypes.byref(f)),
              "ccm_header_decode_fx")
        fx = int(f.value)
    elif order == "C":
        check(lib.ccm_header_decode(hdr, ctypes.byref(d)), "ccm_header_decode")
    else:
        check(lib.ccm_header_decode_cm(hdr, ctypes.byref(d)), "ccm_header_decode_cm")
    nbytes = 8 * int(d.words)
    if len(blob) != 64 + nbytes:
        raise CcmError(E_INVAL, "from_serialized: payload length")
    m = CMatrix(d, device=device, order=order)
    m.frac_bits = fx
    m.payload.zero_()
    host = torch.frombuffer(bytearray(blob[64:]), dtype=torch.uint8)
    m.payload[:nbytes].copy_(host)
    return m


def compress(dense: torch.Tensor, stream=None, order: str = "C") -> CMatrix:
    """SM-compress a 2-D int32/int64 device tensor (range pass, then packing),
    unravelled by row (order "C") or by column (order "F")."""
    t = _device_tensor(dense, "dense")
    if t.dim() != 2:
        raise ValueError("2-D tensor expected")
    if order not in ("C", "F"):
        raise ValueError("order must be 'C' or 'F'")
    code = _dtype_code(t)
    s = _stream(stream)
    d = Desc()
    r, c = (t.shape[0], t.shape[1]) if order == "C" else (t.shape[1], t.shape[0])
    check(lib.ccm_compress_plan(_ptr(t), code, r, c, ctypes.byref(d), s), "ccm_compress_plan")
    m = CMatrix(d, device=t.device, order=order)
    if order == "C":
        check(lib.ccm_compress(_ptr(t), code, ctypes.byref(m.desc), s), "ccm_compress")
    else:
        check(lib.ccm_compress_cm(_ptr(t), code, ctypes.byref(m.desc), s), "ccm_compress_cm")
    return m


def decompress(m: CMatrix, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The dense int64 matrix.  For order "F" the kernel writes the transpose
    row by row and the result is its transposed view (out, if given, receives
    the transpose: shape cols x rows)."""
    if out is None:
        out = torch.empty((m.desc.rows, m.desc.cols), dtype=torch.int64, device=m.payload.device)
    elif out.dtype != torch.int64 or out.numel() != m.rows * m.cols or not out.is_contiguous():
        raise CcmError(E_INVAL, "decompress: out")
    check(lib.ccm_decompress(ctypes.byref(m.desc), _ptr(out), _stream(stream)), "ccm_decompress")
    return out if m.order == "C" else out.view(m.desc.rows, m.desc.cols).t()


def get(m: CMatrix, i: int, j: int, stream=None) -> int:
    v = ctypes.c_int64()
    if m.order == "F":
        i, j = j, i
    check(lib.ccm_get(ctypes.byref(m.desc), i, j, ctypes.byref(v), _stream(stream)), "ccm_get")
    return int(v.value)


def gather(m: CMatrix, ii: torch.Tensor, jj: torch.Tensor, stream=None, sync: bool = True):
    """Elements (ii[t], jj[t]); returns (values, any_out_of_range).  With
    sync=False the second item is the device flag tensor (no host wait)."""
    ii = _device_tensor(ii.to(torch.int64), "ii")
    jj = _device_tensor(jj.to(torch.int64), "jj")
    if m.order == "F":
        ii, jj = jj, ii
    out = torch.empty(ii.numel(), dtype=torch.int64, device=ii.device)
    bad = torch.zeros(1, dtype=torch.int32, device=ii.device)
    check(lib.ccm_gather(ctypes.byref(m.desc), _ptr(ii), _ptr(jj), ii.numel(), _ptr(out),
                         _ptr(bad), _stream(stream)), "ccm_gather")
    return out, (bool(bad.item()) if sync else bad)


def add(a: CMatrix, b: CMatrix, stream=None, onepass: bool = True) -> CMatrix:
    """C = A + B; both operands in the same order (the result keeps it).
    onepass: ccm_add_onepass (packs at the width the headers bound while the
    exact range is reduced); otherwise ccm_add_plan then ccm_add."""
    if a.order != b.order:
        raise CcmError(E_UNSUPPORTED, "add: operands unravelled in different orders")
    if a.frac_bits != b.frac_bits:
        raise CcmError(E_UNSUPPORTED, "add: operands in different fixed-point scales")
    c = _add(a, b, stream, onepass)
    c.frac_bits = a.frac_bits
    return c


def _add(a: CMatrix, b: CMatrix, stream, onepass: bool) -> CMatrix:
    s = _stream(stream)
    d = Desc()
    if onepass:
        if a.shape != b.shape:
            raise CcmError(E_SHAPE, "add: operand shapes differ")
        cap = int(lib.ccm_add_capacity(ctypes.byref(a.desc), ctypes.byref(b.desc)))
        if cap == 0:
            raise CcmError(E_INVAL, "ccm_add_capacity: invalid operands")
        payload = torch.empty(cap, dtype=torch.uint8, device=a.payload.device)
        d.payload = payload.data_ptr()
        check(lib.ccm_add_onepass(ctypes.byref(a.desc), ctypes.byref(b.desc), ctypes.byref(d),
                                  s), "ccm_add_onepass")
        # past the final width's capacity the buffer may hold the first pack's words
        keep = int(lib.ccm_payload_capacity(d.rows, d.cols, d.bits))
        return CMatrix(d, payload[:keep], order=a.order)
    check(lib.ccm_add_plan(ctypes.byref(a.desc), ctypes.byref(b.desc), ctypes.byref(d), s),
          "ccm_add_plan")
    c = CMatrix(d, device=a.payload.device, order=a.order)
    check(lib.ccm_add(ctypes.byref(a.desc), ctypes.byref(b.desc), ctypes.byref(c.desc), s),
          "ccm_add")
    return c


def scale(a: CMatrix, s_: int, stream=None) -> CMatrix:
    d = Desc()
    check(lib.ccm_scale_plan(ctypes.byref(a.desc), s_, ctypes.byref(d)), "ccm_scale_plan")
    c = CMatrix(d, device=a.payload.device, order=a.order)
    check(lib.ccm_scale(ctypes.byref(a.desc), s_, ctypes.byref(c.desc), _stream(stream)),
          "ccm_scale")
    c.frac_bits = a.frac_bits
    return c


def _mv_call(a: CMatrix, transposed: bool):
    """The C entry point computing y = A x (transposed False) or y = A^T x on
    a's stream: a row-major stream runs them directly, a column-major one (the
    row-major stream of A^T) swaps them."""
    row_major_op = transposed == (a.order == "C")
    return (lib.ccm_matvec_t, "ccm_matvec_t") if row_major_op else (lib.ccm_matvec, "ccm_matvec")


# Largest scratch allocated for the split partial sums of y = A^T x; past it
# the splits add with atomics instead.
_MVT_SCRATCH_MAX = 256 << 20


def _mv_args(a: CMatrix, x, y, stream, transposed: bool):
    """The C entry point and its arguments for y = A x (transposed False) or
    y = A^T x; ccm_matvec_t gets scratch for its split partial sums (returned
    too: it must live until the launch completes)."""
    fn, name = _mv_call(a, transposed)
    args = [ctypes.byref(a.desc), _ptr(x), _dtype_code(x), _ptr(y)]
    scratch = None
    if name == "ccm_matvec_t":
        nb = int(lib.ccm_matvec_t_scratch_bytes(ctypes.byref(a.desc)))
        if 0 < nb <= _MVT_SCRATCH_MAX:
            scratch = torch.empty(nb // 8, dtype=torch.int64, device=x.device)
            args += [_ptr(scratch), nb]
        else:
            args += [None, 0]
    args.append(_stream(stream))
    return fn, name, tuple(args), scratch


def _mv(a: CMatrix, x, y, stream, transposed: bool):
    nin, nout = (a.rows, a.cols) if transposed else (a.cols, a.rows)
    x = _device_tensor(x, "x")
    if x.numel() != nin:
        raise CcmError(E_SHAPE, "matvec")
    if y is None:
        y = torch.empty(nout, dtype=torch.int64, device=x.device)
    elif y.dtype != torch.int64 or y.numel() != nout or not y.is_contiguous():
        raise CcmError(E_INVAL, "matvec: y")
    fn, name, args, scratch = _mv_args(a, x, y, stream, transposed)
    check(fn(*args), name)
    if scratch is not None and stream is not None:
        scratch.record_stream(stream)  # freed for reuse only after that stream's work
    return y


def matvec(a: CMatrix, x: torch.Tensor, y: torch.Tensor | None = None, stream=None):
    """y = A x (int64, modulo 2^64); x is an int32 or int64 device vector."""
    return _mv(a, x, y, stream, transposed=False)


def matvec_t(a: CMatrix, x: torch.Tensor, y: torch.Tensor | None = None, stream=None):
    """y = A^T x (int64, modulo 2^64); x has one value per row of A."""
    return _mv(a, x, y, stream, transposed=True)


def matvec_launcher(a: CMatrix, x: torch.Tensor, y: torch.Tensor, stream=None,
                    transposed: bool = False):
    """Marshals the arguments of y = A x (y = A^T x when transposed) once and
    returns a callable that launches it with no further Python work (for
    back-to-back launches whose kernels are shorter than the per-call
    marshalling).  a, x and y must stay alive while the callable is used."""
    nin, nout = (a.rows, a.cols) if transposed else (a.cols, a.rows)
    x = _device_tensor(x, "x")
    if x.numel() != nin:
        raise CcmError(E_SHAPE, "matvec")
    if y.dtype != torch.int64 or y.numel() != nout or not y.is_contiguous():
        raise CcmError(E_INVAL, "matvec: y")
    fn, name, args, scratch = _mv_args(a, x, y, stream, transposed)

    def launch():
        _ = scratch  # the scratch lives as long as the callable
        rc = fn(*args)
        if rc != 0:
            raise CcmError(rc, name)
    return launch


def matmul_scratch_bytes(a: CMatrix, b: CMatrix) -> int:
    _row_major(a, "matmul")
    _row_major(b, "matmul")
    return int(lib.ccm_matmul_scratch_bytes(ctypes.byref(a.desc), ctypes.byref(b.desc)))


def matmul_plan(a: CMatrix, b: CMatrix, scratch: torch.Tensor | None = None, stream=None):
    """Range pass of C = A B: computes C into scratch and returns (C, scratch), C
    allocated at its final width but not yet packed."""
    _row_major(a, "matmul")
    _row_major(b, "matmul")
    if a.cols != b.rows:
        raise CcmError(E_SHAPE, "matmul")
    need = matmul_scratch_bytes(a, b)
    if need == 0:
        # invalid descriptors or the overflow bound: let the plan report which
        need = 8
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=a.payload.device)
    d = Desc()
    check(lib.ccm_matmul_plan(ctypes.byref(a.desc), ctypes.byref(b.desc), ctypes.byref(d),
                              _ptr(scratch), scratch.numel(), _stream(stream)), "ccm_matmul_plan")
    return CMatrix(d, device=a.payload.device), scratch


def matmul_pack(a: CMatrix, b: CMatrix, c: CMatrix, scratch: torch.Tensor, stream=None):
    """Packing pass of C = A B from the scratch its plan filled."""
    check(lib.ccm_matmul(ctypes.byref(a.desc), ctypes.byref(b.desc), ctypes.byref(c.desc),
                         _ptr(scratch), scratch.numel(), _stream(stream)), "ccm_matmul")
    return c


def matmul(a: CMatrix, b: CMatrix, scratch: torch.Tensor | None = None, stream=None) -> CMatrix:
    c, scratch = matmul_plan(a, b, scratch, stream)
    c = matmul_pack(a, b, c, scratch, stream)
    if a.frac_bits is not None or b.frac_bits is not None:
        c.frac_bits = (a.frac_bits or 0) + (b.frac_bits or 0)
    return c


# ---- results whose width stays on the device ------------------------------

def async_ws(device="cuda") -> torch.Tensor:
    """A workspace for one asynchronous result in flight (the device writes
    the result's header fields into its first 64 bytes)."""
    return torch.empty(int(lib.ccm_async_ws_bytes()), dtype=torch.uint8, device=device)


class Pending:
    """A matrix-valued result enqueued with ccm_add_async / ccm_matmul_async.
    Its header fields stay on the device until the work completes; `done()`
    polls without blocking, `get()` waits and returns the CMatrix."""

    def __init__(self, payload: torch.Tensor, ws: torch.Tensor, host: torch.Tensor, stream,
                 order: str = "C", keep=()):
        self.payload, self.ws, self.host, self.order = payload, ws, host, order
        self._keep = keep  # inputs that must live until the work completes
        self.event = torch.cuda.Event()
        self.event.record(stream)
        self._mat = None

    def done(self) -> bool:
        return self.event.query()

    def get(self) -> CMatrix:
        if self._mat is None:
            self.event.synchronize()
            r = Result.from_buffer_copy(bytes(self.host.numpy().tobytes()))
            d = Desc()
            check(lib.ccm_result_desc(ctypes.byref(r), ctypes.c_void_p(self.payload.data_ptr()),
                                      ctypes.byref(d)), "ccm_result_desc")
            keep = int(lib.ccm_payload_capacity(d.rows, d.cols, d.bits))
            self._mat = CMatrix(d, self.payload[:keep], order=self.order)
            self._keep = ()
        return self._mat


def _pending(payload, ws, host, stream, order, keep):
    s = stream if stream is not None else torch.cuda.current_stream()
    if host is None:
        host = torch.empty(64, dtype=torch.uint8, pin_memory=True)
    with torch.cuda.stream(s):
        host.copy_(ws[:64], non_blocking=True)
    return Pending(payload, ws, host, s, order, keep)


def add_async(a: CMatrix, b: CMatrix, ws: torch.Tensor | None = None,
              host: torch.Tensor | None = None, stream=None) -> Pending:
    """C = A + B with no host wait (ccm_add_async); host: optional pinned
    64-byte buffer that receives the result's header fields."""
    if a.order != b.order:
        raise CcmError(E_UNSUPPORTED, "add: operands unravelled in different orders")
    if a.shape != b.shape:
        raise CcmError(E_SHAPE, "add: operand shapes differ")
    cap = int(lib.ccm_add_capacity(ctypes.byref(a.desc), ctypes.byref(b.desc)))
    if cap == 0:
        raise CcmError(E_INVAL, "ccm_add_capacity: invalid operands")
    payload = torch.empty(cap, dtype=torch.uint8, device=a.payload.device)
    ws = async_ws(a.payload.device) if ws is None else ws
    check(lib.ccm_add_async(ctypes.byref(a.desc), ctypes.byref(b.desc), _ptr(payload), cap,
                            _ptr(ws), _stream(stream)), "ccm_add_async")
    return _pending(payload, ws, host, stream, a.order, (a, b))


def matmul_capacity(a: CMatrix, b: CMatrix) -> int:
    _row_major(a, "matmul")
    _row_major(b, "matmul")
    return int(lib.ccm_matmul_capacity(ctypes.byref(a.desc), ctypes.byref(b.desc)))


def matmul_async(a: CMatrix, b: CMatrix, scratch: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None, payload: torch.Tensor | None = None,
                 host: torch.Tensor | None = None, stream=None) -> Pending:
    """C = A B with no host wait (ccm_matmul_async)."""
    _row_major(a, "matmul")
    _row_major(b, "matmul")
    if a.cols != b.rows:
        raise CcmError(E_SHAPE, "matmul")
    cap = matmul_capacity(a, b)
    need = matmul_scratch_bytes(a, b)
    if cap == 0 or need == 0:
        raise CcmError(E_OVERFLOW, "matmul: operands past the overflow bound")
    dev = a.payload.device
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=dev)
    if payload is None or payload.numel() < cap:
        payload = torch.empty(cap, dtype=torch.uint8, device=dev)
    ws = async_ws(dev) if ws is None else ws
    check(lib.ccm_matmul_async(ctypes.byref(a.desc), ctypes.byref(b.desc), _ptr(payload),
                               payload.numel(), _ptr(scratch), scratch.numel(), _ptr(ws),
                               _stream(stream)), "ccm_matmul_async")
    return _pending(payload, ws, host, stream, "C", (a, b, scratch))


class VlbMatrix:
    """A Method 2 (variable length blocks) matrix: descriptor, device stream
    and device index (row starts, group offsets)."""

    def __init__(self, desc: VlbDesc, index: torch.Tensor, payload: torch.Tensor | None = None):
        self.desc = desc
        self.index = index
        if payload is None:
            cap = int(lib.ccm_vlb_payload_capacity(desc.nbits))
            payload = torch.empty(cap, dtype=torch.uint8, device=index.device)
        self.payload = payload
        self.desc.payload = payload.data_ptr()
        # fixed-point matrices (floats, Conclusion): the values are q 2^-frac_bits
        self.frac_bits = None
        self.desc.index = index.data_ptr()

    rows = property(lambda self: int(self.desc.rows))
    cols = property(lambda self: int(self.desc.cols))
    vmin = property(lambda self: int(self.desc.vmin))
    vmax = property(lambda self: int(self.desc.vmax))
    k = property(lambda self: int(self.desc.k))
    is_signed = property(lambda self: bool(self.desc.is_signed))
    nbits = property(lambda self: int(self.desc.nbits))
    words = property(lambda self: int(self.desc.words))
    gmax = property(lambda self: int(self.desc.gmax))

    @property
    def shape(self):
        return (self.rows, self.cols)

    @property
    def index_bytes(self) -> int:
        return int(self.index.numel())

    def payload_words(self) -> torch.Tensor:
        """The canonical payload (floor(nbits/64) + 1 bitstrings) as int64 (host)."""
        torch.cuda.current_stream().synchronize()
        return self.payload[: 8 * self.words].view(torch.int64).cpu()

    def row_bits(self) -> torch.Tensor:
        """row_bit[0..rows] (host int64 copy of the index's uint64 row starts)."""
        torch.cuda.current_stream().synchronize()
        return self.index[: 8 * (self.rows + 1)].view(torch.int64).cpu()

    def group_offsets(self) -> torch.Tensor:
        """grp_off[rows][ceil(cols/32)] (host int64 copy)."""
        torch.cuda.current_stream().synchronize()
        off = ((self.rows + 1) * 8 + 255) // 256 * 256
        ngr = (self.cols + 31) // 32
        g = self.index[off: off + 4 * self.rows * ngr].view(torch.int32).cpu()
        return (g.to(torch.int64) & 0xFFFFFFFF).view(self.rows, ngr)

    def __repr__(self):
        return (f"VlbMatrix({self.rows}x{self.cols}, k={self.k}, signed={self.is_signed}, "
                f"nbits={self.nbits})")


def vlb_compress(dense: torch.Tensor, stream=None) -> VlbMatrix:
    """Method 2-compress a 2-D int32/int64 device tensor (range pass, index
    passes, then packing)."""
    t = _device_tensor(dense, "dense")
    if t.dim() != 2:
        raise ValueError("2-D tensor expected")
    code = _dtype_code(t)
    s = _stream(stream)
    rows, cols = t.shape
    nidx = int(lib.ccm_vlb_index_bytes(rows, cols))
    if nidx == 0:
        raise CcmError(E_INVAL, "vlb_compress: shape")
    index = torch.empty(nidx, dtype=torch.uint8, device=t.device)
    d = VlbDesc()
    check(lib.ccm_vlb_compress_plan(_ptr(t), code, rows, cols, _ptr(index), ctypes.byref(d), s),
          "ccm_vlb_compress_plan")
    m = VlbMatrix(d, index)
    check(lib.ccm_vlb_compress(_ptr(t), code, ctypes.byref(m.desc), s), "ccm_vlb_compress")
    return m


def vlb_decompress(m: VlbMatrix, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if out is None:
        out = torch.empty((m.rows, m.cols), dtype=torch.int64, device=m.payload.device)
    elif out.dtype != torch.int64 or out.numel() != m.rows * m.cols or not out.is_contiguous():
        raise CcmError(E_INVAL, "vlb_decompress: out")
    check(lib.ccm_vlb_decompress(ctypes.byref(m.desc), _ptr(out), _stream(stream)),
          "ccm_vlb_decompress")
    return out


def vlb_get(m: VlbMatrix, i: int, j: int, stream=None) -> int:
    v = ctypes.c_int64()
    check(lib.ccm_vlb_get(ctypes.byref(m.desc), i, j, ctypes.byref(v), _stream(stream)),
          "ccm_vlb_get")
    return int(v.value)


def vlb_matvec(m: VlbMatrix, x: torch.Tensor, y: torch.Tensor | None = None, stream=None):
    x = _device_tensor(x, "x")
    if x.numel() != m.cols:
        raise CcmError(E_SHAPE, "vlb_matvec: x")
    if y is None:
        y = torch.empty(m.rows, dtype=torch.int64, device=x.device)
    elif y.dtype != torch.int64 or y.numel() != m.rows or not y.is_contiguous():
        raise CcmError(E_INVAL, "vlb_matvec: y")
    check(lib.ccm_vlb_matvec(ctypes.byref(m.desc), _ptr(x), _dtype_code(x), _ptr(y),
                             _stream(stream)), "ccm_vlb_matvec")
    return y


def vlb_matvec_launcher(m: VlbMatrix, x: torch.Tensor, y: torch.Tensor, stream=None):
    """A zero-argument callable that enqueues y = A x with every argument
    marshalled once (for timing loops)."""
    x = _device_tensor(x, "x")
    if x.numel() != m.cols or y.dtype != torch.int64 or y.numel() != m.rows:
        raise CcmError(E_SHAPE, "vlb_matvec_launcher")
    fn = lib.ccm_vlb_matvec
    args = (ctypes.byref(m.desc), _ptr(x), _dtype_code(x), _ptr(y), _stream(stream))

    def launch():
        check(fn(*args), "ccm_vlb_matvec")

    return launch


def method_info(dense: torch.Tensor, stream=None) -> dict:
    """Both methods' exact bit counts and efficiencies (Eq. 15, Eq. 17) and the
    method using fewer bits (1 on a tie), from one pass over dense."""
    t = _device_tensor(dense, "dense")
    if t.dim() != 2:
        raise ValueError("2-D tensor expected")
    info = MethodInfo()
    check(lib.ccm_method_plan(_ptr(t), _dtype_code(t), t.shape[0], t.shape[1],
                              ctypes.byref(info), _stream(stream)), "ccm_method_plan")
    return {f: getattr(info, f) for f, _ in MethodInfo._fields_ if f != "reserved"}


def compress_auto(dense: torch.Tensor, stream=None):
    """Compress with the method that uses fewer bits: a CMatrix (Method 1) or a
    VlbMatrix (Method 2)."""
    info = method_info(dense, stream)
    return compress(dense, stream) if info["method"] == 1 else vlb_compress(dense, stream)


def fill_uniform(t: torch.Tensor, lo: int, hi: int, seed: int, stream_id: int = 0,
                 start: int = 0, stream=None) -> torch.Tensor:
    """Fill a device int32/int64 tensor with seeded SplitMix64 draws in [lo, hi)."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("contiguous device tensor expected")
    check(lib.ccm_fill_uniform(_ptr(t), _dtype_code(t), t.numel(), lo, hi, seed, stream_id,
                               start, _stream(stream)), "ccm_fill_uniform")
    return t


def generate(rows: int, cols: int, lo: int, hi: int, seed: int, stream_id: int = 0,
             device="cuda", stream=None) -> CMatrix:
    """Compressed matrix of seeded draws, packed on the device without a dense copy."""
    s = _stream(stream)
    d = Desc()
    check(lib.ccm_generate_plan(rows, cols, lo, hi, seed, stream_id, ctypes.byref(d), s),
          "ccm_generate_plan")
    m = CMatrix(d, device=device)
    check(lib.ccm_generate(ctypes.byref(m.desc), lo, hi, seed, stream_id, s), "ccm_generate")
    return m


from .batch import Batch, DynBatch  # noqa: E402


# ---- floats in fixed point (Conclusion) -----------------------------------
#
# A float matrix is stored as q = round-half-to-even(v 2^f) (one f per matrix)
# packed by Method 1; every operation is then the exact integer one on q, and
# float results are the exact integer results converted back (include/ccm.h).

def float_absmax(v: torch.Tensor, stream=None) -> float:
    """Largest |v| of a float32/float64 device tensor (exact); CcmError
    E_RANGE for NaN or infinity."""
    t = _device_tensor(v, "v")
    a = ctypes.c_double()
    check(lib.ccm_float_absmax(_ptr(t), _float_code(t), t.numel(), ctypes.byref(a),
                               _stream(stream)), "ccm_float_absmax")
    return float(a.value)


def float_frac_bits(absmax: float, sig_bits: int) -> int:
    """Fraction bits keeping sig_bits significant bits of the largest
    magnitude: sig_bits - 1 - floor(log2 absmax)."""
    f = ctypes.c_int32()
    check(lib.ccm_float_frac_bits(float(absmax), sig_bits, ctypes.byref(f)),
          "ccm_float_frac_bits")
    return int(f.value)


def quantize(v: torch.Tensor, frac_bits: int, out: torch.Tensor | None = None, stream=None,
             dtype=torch.int64):
    """(q, qmin, qmax): q = round-half-to-even(v 2^frac_bits) as int64 (or
    int32), same shape, and its exact extremes."""
    t = _device_tensor(v, "v")
    if out is None:
        out = torch.empty(t.shape, dtype=dtype, device=t.device)
    elif out.numel() != t.numel() or not out.is_contiguous():
        raise CcmError(E_INVAL, "quantize: out")
    lo, hi = ctypes.c_int64(), ctypes.c_int64()
    check(lib.ccm_quantize(_ptr(t), _float_code(t), t.numel(), frac_bits, _ptr(out),
                           _dtype_code(out), ctypes.byref(lo), ctypes.byref(hi),
                           _stream(stream)), "ccm_quantize")
    return out, int(lo.value), int(hi.value)


def dequantize(q: torch.Tensor, frac_bits: int, dtype=torch.float64,
               out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """q 2^-frac_bits as float64 or float32 (one rounding to double, the exact
    scaling, and for float32 one more rounding)."""
    t = _device_tensor(q, "q")
    if t.dtype != torch.int64:
        raise TypeError("int64 tensor expected")
    if out is None:
        out = torch.empty(t.shape, dtype=dtype, device=t.device)
    elif out.numel() != t.numel() or not out.is_contiguous():
        raise CcmError(E_INVAL, "dequantize: out")
    check(lib.ccm_dequantize(_ptr(t), t.numel(), frac_bits, _float_code(out), _ptr(out),
                             _stream(stream)), "ccm_dequantize")
    return out


def _keep(t: torch.Tensor, stream) -> None:
    """A temporary read by work enqueued on `stream`: tell the caching
    allocator, so its memory is not handed out again before that work ran."""
    if stream is not None:
        t.record_stream(stream)


def _frac_bits_of(v: torch.Tensor, sig_bits, frac_bits, stream) -> int:
    if (sig_bits is None) == (frac_bits is None):
        raise ValueError("give exactly one of sig_bits and frac_bits")
    if frac_bits is not None:
        return int(frac_bits)
    return float_frac_bits(float_absmax(v, stream), sig_bits)


def compress_float(dense: torch.Tensor, sig_bits: int | None = None,
                   frac_bits: int | None = None, stream=None) -> CMatrix:
    """A 2-D float32/float64 device tensor in fixed point: quantized at
    frac_bits (or at the fraction bits that keep sig_bits significant bits of
    its largest magnitude) and SM-packed like an integer matrix: one pass
    yields the quantized values' exact range, a second packs them straight
    from the floats."""
    t = _device_tensor(dense, "dense")
    if t.dim() != 2:
        raise ValueError("2-D tensor expected")
    f = _frac_bits_of(t, sig_bits, frac_bits, stream)
    lo, hi = ctypes.c_int64(), ctypes.c_int64()
    check(lib.ccm_quantize(_ptr(t), _float_code(t), t.numel(), f, None, I64, ctypes.byref(lo),
                           ctypes.byref(hi), _stream(stream)), "ccm_quantize")
    b, sgn = width(lo.value, hi.value)
    d = Desc()
    d.rows, d.cols, d.vmin, d.vmax = t.shape[0], t.shape[1], lo.value, hi.value
    d.bits, d.is_signed, d.words = b, 1 if sgn else 0, words(t.shape[0], t.shape[1], b)
    m = CMatrix(d, device=t.device)
    check(lib.ccm_compress_fx(_ptr(t), _float_code(t), f, ctypes.byref(m.desc),
                              _stream(stream)), "ccm_compress_fx")
    _keep(t, stream)
    m.frac_bits = f
    return m


def decompress_float(m: CMatrix, dtype=torch.float64, stream=None) -> torch.Tensor:
    """The fixed-point matrix as floats: q decoded, then q 2^-frac_bits."""
    if m.frac_bits is None:
        raise CcmError(E_INVAL, "decompress_float: not a fixed-point matrix")
    q = decompress(m, stream=stream)
    out = torch.empty(q.shape, dtype=dtype, device=q.device)
    q = q.contiguous()
    dequantize(q, m.frac_bits, dtype, out=out, stream=stream)
    _keep(q, stream)
    return out


def matvec_float(m: CMatrix, x: torch.Tensor, x_sig_bits: int | None = None,
                 x_frac_bits: int | None = None, stream=None) -> torch.Tensor:
    """y = V x for a fixed-point V: x quantized at x_frac_bits (or keeping
    x_sig_bits significant bits), the exact integer matvec, and y converted
    back at frac_bits + x_frac_bits, as float64.  CcmError E_OVERFLOW when
    cols * max|q| * max|x_q| >= 2^63 (the integer sums could wrap)."""
    if m.frac_bits is None:
        raise CcmError(E_INVAL, "matvec_float: not a fixed-point matrix")
    t = _device_tensor(x, "x")
    g = _frac_bits_of(t, x_sig_bits, x_frac_bits, stream)
    # with at most 31 significant bits kept, |x_q| <= 2^31 - 1 after rounding
    # is not guaranteed (2^31 itself can appear), so int32 only up to 30
    narrow = x_sig_bits is not None and x_sig_bits <= 30
    xq, xlo, xhi = quantize(t, g, stream=stream, dtype=torch.int32 if narrow else torch.int64)
    amax = max(abs(m.vmin), abs(m.vmax))
    if m.cols * amax * max(abs(xlo), abs(xhi)) >= (1 << 63):
        raise CcmError(E_OVERFLOW, "matvec_float: the integer sums could leave int64")
    y = matvec(m, xq, stream=stream)
    out = dequantize(y, m.frac_bits + g, torch.float64, stream=stream)
    _keep(xq, stream)
    _keep(y, stream)
    return out
