"""Seeded synthetic inputs for the compressed-matrix workloads.

This module only draws random integers; it holds none of the compression
method's arithmetic, so both the GPU library's tests and the CPU oracle may
use it.

Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-style: output number ``ctr`` of
the sequence that starts at state ``seed`` is

    z = seed + (ctr + 1) * 0x9E3779B97F4A7C15            (mod 2^64)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    h = z ^ (z >> 31)

so any element can be regenerated on its own.  A draw in ``[lo, hi)`` with
``span = hi - lo <= 2^32`` is ``lo + (((h >> 32) * span) >> 32)`` (Lemire's
multiply-shift on the top 32 bits; exact for power-of-two spans).  The GPU
library's fill kernels implement the same definition independently; a test
checks that both produce identical values.

Counters: element ``idx`` of stream ``s`` uses ``ctr = (s << 40) + idx``
(streams hold fewer than 2^40 elements).

Seeds: ``1303027000 + 10 * workload + operand`` (operand 0 = A, 1 = B, 2 = x).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
SEED_BASE = 1303027000
STREAM_SHIFT = 40


def seed_for(workload: int, operand: int) -> int:
    return SEED_BASE + 10 * workload + operand


def splitmix64(seed: int, ctr: np.ndarray) -> np.ndarray:
    """Output number ``ctr`` (uint64 array) of the SplitMix64 sequence from ``seed``."""
    c = np.asarray(ctr, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & (2**64 - 1)) + (c + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, stream: int, start: int, count: int, lo: int, hi: int) -> np.ndarray:
    """Draws ``start .. start+count-1`` of stream ``stream``, uniform in [lo, hi)."""
    span = hi - lo
    if not (1 <= span <= 2**32):
        raise ValueError("span must be in [1, 2^32]")
    ctr = (np.uint64(stream) << np.uint64(STREAM_SHIFT)) + np.arange(start, start + count,
                                                                      dtype=np.uint64)
    h = splitmix64(seed, ctr)
    with np.errstate(over="ignore"):
        off = ((h >> np.uint64(32)) * np.uint64(span)) >> np.uint64(32)
    return (off.astype(np.int64) + np.int64(lo)).astype(np.int64)


def uniform_at(seed: int, stream: int, idx: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Draws number ``idx`` (any int64 array) of stream ``stream``, uniform in
    [lo, hi): the same values ``uniform`` gives at those positions."""
    span = hi - lo
    if not (1 <= span <= 2**32):
        raise ValueError("span must be in [1, 2^32]")
    ctr = (np.uint64(stream) << np.uint64(STREAM_SHIFT)) + np.asarray(idx, dtype=np.uint64)
    h = splitmix64(seed, ctr)
    with np.errstate(over="ignore"):
        off = ((h >> np.uint64(32)) * np.uint64(span)) >> np.uint64(32)
    return (off.astype(np.int64) + np.int64(lo)).astype(np.int64)


def uniform_matrix(seed: int, stream: int, rows: int, cols: int, lo: int, hi: int) -> np.ndarray:
    return uniform(seed, stream, 0, rows * cols, lo, hi).reshape(rows, cols)


def matrix_rows(seed: int, stream: int, cols: int, r0: int, r1: int, lo: int, hi: int):
    """Rows [r0, r1) of ``uniform_matrix(seed, stream, rows, cols, lo, hi)``."""
    return uniform(seed, stream, r0 * cols, (r1 - r0) * cols, lo, hi).reshape(r1 - r0, cols)


# ---------------------------------------------------------------------------
# Workloads (shapes, ranges and seeds)
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class MatrixSpec:
    """A seeded uniform matrix: values ``uniform(seed, stream, ., ., lo, hi)``."""
    rows: int
    cols: int
    lo: int
    hi: int
    seed: int
    stream: int = 0

    def dense(self) -> np.ndarray:
        return uniform_matrix(self.seed, self.stream, self.rows, self.cols, self.lo, self.hi)

    def rows_slice(self, r0: int, r1: int) -> np.ndarray:
        return matrix_rows(self.seed, self.stream, self.cols, r0, r1, self.lo, self.hi)

    def column(self, j: int) -> np.ndarray:
        """Column j (rows values)."""
        idx = np.arange(self.rows, dtype=np.int64) * self.cols + j
        return uniform_at(self.seed, self.stream, idx, self.lo, self.hi)


@dataclass(frozen=True)
class VectorSpec:
    n: int
    lo: int
    hi: int
    seed: int
    stream: int = 0

    def dense(self) -> np.ndarray:
        return uniform(self.seed, self.stream, 0, self.n, self.lo, self.hi)


# Plain method, small: 256x256 in [0, 2^10), int64 x in [0, 1000), scalar 7.
def small_plain(n: int = 256):
    a = MatrixSpec(n, n, 0, 1 << 10, seed_for(1, 0))
    b = MatrixSpec(n, n, 0, 1 << 10, seed_for(1, 1))
    x = VectorSpec(n, 0, 1000, seed_for(1, 2))
    return a, b, x, 7


SWEEP_WIDTHS = (1, 3, 7, 12, 17, 31)


# Bandwidth sweep: n x n in [0, 2^k) or [-2^(k-1), 2^(k-1)); int32 x in [-2^15, 2^15).
def sweep(k: int, signed: bool, n: int = 16384):
    lo, hi = ((-(1 << (k - 1)), 1 << (k - 1)) if signed else (0, 1 << k))
    stream = 2 * k + (1 if signed else 0)
    a = MatrixSpec(n, n, lo, hi, seed_for(2, 0), stream)
    b = MatrixSpec(n, n, lo, hi, seed_for(2, 1), stream)
    x = VectorSpec(n, -(1 << 15), 1 << 15, seed_for(2, 2))
    return a, b, x, 7


# Dense compressed GEMM: A in [0, 2^6), B in [-2^3, 2^3).
def dense_gemm(n: int = 8192, k: int | None = None, m: int | None = None):
    k = n if k is None else k
    m = n if m is None else m
    a = MatrixSpec(n, k, 0, 1 << 6, seed_for(3, 0))
    b = MatrixSpec(k, m, -(1 << 3), 1 << 3, seed_for(3, 1))
    return a, b


# Floats in fixed point: an n x n float32 matrix v = m 2^e with m uniform in
# [-2^23, 2^23) and e uniform in [-20, 0] (exact float32 values spread over
# six decimal orders of magnitude), and x = m' 2^-23 with m' uniform in
# [-2^23, 2^23).  Returns (mantissas, exponents, x mantissas); the floats are
# formed from them exactly (ldexp) wherever they are needed.
def float_matrix(n: int = 16384):
    m = MatrixSpec(n, n, -(1 << 23), 1 << 23, seed_for(7, 0), 0)
    e = MatrixSpec(n, n, -20, 1, seed_for(7, 0), 1)
    x = VectorSpec(n, -(1 << 23), 1 << 23, seed_for(7, 2))
    return m, e, x


@dataclass(frozen=True)
class BatchItem:
    a: MatrixSpec
    x: VectorSpec
    bits: int


# Batched: rows, cols uniform in [32, 2048], width uniform in 1..24, values in
# [0, 2^width); one int32 x per matrix in [-2^15, 2^15).
def batched(count: int = 4096, lo_dim: int = 32, hi_dim: int = 2048, max_bits: int = 24):
    seed = seed_for(4, 0)
    rows = uniform(seed, 0, 0, count, lo_dim, hi_dim + 1)
    cols = uniform(seed, 1, 0, count, lo_dim, hi_dim + 1)
    bits = uniform(seed, 2, 0, count, 1, max_bits + 1)
    items = []
    for t in range(count):
        b = int(bits[t])
        items.append(BatchItem(
            MatrixSpec(int(rows[t]), int(cols[t]), 0, 1 << b, seed_for(4, 1), 16 + t),
            VectorSpec(int(cols[t]), -(1 << 15), 1 << 15, seed_for(4, 2), 16 + t), b))
    return items


@dataclass(frozen=True)
class PoolMatrix:
    rows: int
    cols: int
    bits: int
    spec: MatrixSpec


# Serving pool: n = floor(10^U(4, 9)) elements, rows = floor(sqrt(n)),
# cols = ceil(n / rows), width uniform in 1..20, values in [0, 2^width); drawn
# until the packed total reaches target_bytes.
def serving_pool(target_bytes: float, max_elems: float = 1e9, max_bits: int = 20,
                 min_exp: float = 4.0):
    seed = seed_for(5, 0)
    max_exp = math.log10(max_elems)
    out, total, t = [], 0, 0
    while total < target_bytes:
        u = uniform(seed, 0, t, 1, 0, 1 << 32)[0] / float(1 << 32)
        n = int(10 ** (min_exp + (max_exp - min_exp) * u))
        n = max(n, 1)
        rows = max(int(math.isqrt(n)), 1)
        cols = -(-n // rows)
        b = int(uniform(seed, 1, t, 1, 1, max_bits + 1)[0])
        spec = MatrixSpec(rows, cols, 0, 1 << b, seed_for(5, 1), 16 + t)
        out.append(PoolMatrix(rows, cols, b, spec))
        total += 64 + 8 * ((rows * cols * b) // 64 + 1)
        t += 1
    return out


# ---------------------------------------------------------------------------
# Method 2 workloads: element bit-lengths drawn from the paper's Beta
# distributions mapped to [1, 64] (Results, "Random Matrix Generation", Eq. 18:
# L = floor(64 x) + 1), then a value of exactly that bit-length.
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class VlbSpec:
    """rows x cols matrix whose element bit-lengths follow
    (1 - w) Beta(a1, b1) + w Beta(a2, b2) on [1, 64] (w = 0: one Beta).

    Element idx draws u = uniform(seed, 3*stream, idx, 0, 2^32); its bit-length
    is L = 1 + #{l in 1..62 : u >= t_l} with t_l = floor(2^32 P(L <= l)), so
    lengths 63 and 64 both give 63 (the largest non-negative int64 length).
    Its value takes the low L-1 bits of r = (h << 32) | g, with h and g draws
    of streams 3*stream + 1 and 3*stream + 2 in [0, 2^32), and sets bit L-1
    (L = 1: the value is r & 1, i.e. 0 or 1)."""
    rows: int
    cols: int
    a1: float
    b1: float
    seed: int
    stream: int = 0
    a2: float = 1.0
    b2: float = 1.0
    w: float = 0.0

    def thresholds(self) -> np.ndarray:
        from scipy.special import betainc
        edges = np.arange(1, 63, dtype=np.float64) / 64.0
        cdf = (1.0 - self.w) * betainc(self.a1, self.b1, edges)
        if self.w:
            cdf = cdf + self.w * betainc(self.a2, self.b2, edges)
        t = np.floor(np.clip(cdf, 0.0, 1.0) * float(1 << 32))
        return np.maximum.accumulate(t.astype(np.uint64))

    def values(self, start: int, count: int) -> np.ndarray:
        u = uniform(self.seed, 3 * self.stream, start, count, 0, 1 << 32).astype(np.uint64)
        L = 1 + np.searchsorted(self.thresholds(), u, side="right").astype(np.int64)
        h = uniform(self.seed, 3 * self.stream + 1, start, count, 0, 1 << 32).astype(np.uint64)
        g = uniform(self.seed, 3 * self.stream + 2, start, count, 0, 1 << 32).astype(np.uint64)
        r = (h << np.uint64(32)) | g
        top = np.left_shift(np.uint64(1), (L - 1).astype(np.uint64))
        v = np.where(L == 1, r & np.uint64(1), top | (r & (top - np.uint64(1))))
        return v.astype(np.int64)

    def rows_slice(self, r0: int, r1: int) -> np.ndarray:
        return self.values(r0 * self.cols, (r1 - r0) * self.cols).reshape(r1 - r0, self.cols)

    def dense(self) -> np.ndarray:
        return self.rows_slice(0, self.rows)

    def dense_device(self, fill_uniform, torch):
        """The same matrix built on the GPU: fill_uniform(tensor, lo, hi, seed,
        stream, start) must draw uniform(seed, stream, start + ., ., lo, hi)
        into an int64 device tensor (the GPU library's generator does)."""
        n = self.rows * self.cols
        dev = torch.device("cuda")
        u = fill_uniform(torch.empty(n, dtype=torch.int64, device=dev), 0, 1 << 32, self.seed,
                         3 * self.stream, 0)
        thr = torch.from_numpy(self.thresholds().astype(np.int64)).to(dev)
        L = 1 + torch.searchsorted(thr, u, right=True)
        del u
        h = fill_uniform(torch.empty(n, dtype=torch.int64, device=dev), 0, 1 << 32, self.seed,
                         3 * self.stream + 1, 0)
        g = fill_uniform(torch.empty(n, dtype=torch.int64, device=dev), 0, 1 << 32, self.seed,
                         3 * self.stream + 2, 0)
        r = torch.bitwise_or(torch.bitwise_left_shift(h, 32), g)
        del h, g
        top = torch.bitwise_left_shift(torch.ones_like(L), L - 1)
        v = torch.where(L == 1, r & 1, top | (r & (top - 1)))
        return v.view(self.rows, self.cols)


# Method 2 bandwidth workloads, n x n: bit-lengths from Beta(1, 32) (short,
# mean about 3 bits), Beta(5, 33) (mean about 9.4 bits) and Beta(1, 1) (uniform
# over 1..64); int32 x in [-2^15, 2^15).
VLB_BETAS = {"beta_1_32": (1.0, 32.0), "beta_5_33": (5.0, 33.0), "beta_1_1": (1.0, 1.0)}


def vlb_sweep(name: str, n: int = 16384):
    a1, b1 = VLB_BETAS[name]
    stream = sorted(VLB_BETAS).index(name)
    a = VlbSpec(n, n, a1, b1, seed_for(6, 0), stream)
    x = VectorSpec(n, -(1 << 15), 1 << 15, seed_for(6, 2), stream)
    return a, x
