"""Floats in fixed point on the GPU against the CPU oracle.

Floats, which the Conclusion allows if some precision is given up, in this
library's reading: q = round-half-to-even(v 2^f), SM-packed like any integer matrix,
every operation exact on q, results converted back.  Quantization (float32
and float64, ties, subnormals, signed zeros, values next to the 2^62 bound),
the error codes, the exact largest magnitude, dequantization (bit patterns of
both float types, scales that make results subnormal), the fixed-point
header and payload, decompress, y = V x, serialization and the scale carried
through add, scale and matmul are compared bit for bit with the oracle.
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import ccm_workloads as W
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "gpu tests need a GPU"
    import paper_1303_0270_amd  # noqa: F401  (fails loudly without libccm.so)


def ccm():
    import paper_1303_0270_amd as c
    return c


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def values(rng, shape, f, dtype=np.float64):
    """Normal values scaled so that |v 2^f| stays below 2^40, with exact ties
    (k + 1/2) 2^-f, zeros of both signs and (for large f) subnormals mixed in."""
    v = np.ldexp(rng.standard_normal(size=shape), int(rng.integers(0, 40)) - f)
    flat = v.reshape(-1)
    k = rng.integers(0, flat.size, size=min(flat.size, 40))
    flat[k[: len(k) // 2]] = np.ldexp(rng.integers(-1000, 1000, size=len(k) // 2) + 0.5, -f)
    flat[k[len(k) // 2:]] = 0.0
    flat[int(rng.integers(0, flat.size))] = -0.0
    if f > 1000:
        flat[int(rng.integers(0, flat.size))] = 5e-324
    return v.astype(dtype)


F_CASES = [0, 3, 12, 30, -4, -30, 200, 1074]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("f", F_CASES)
def test_quantize_matches_oracle(dtype, f):
    c = ccm()
    rng = np.random.default_rng(1000 + f)
    for shape in ((1,), (7,), (1000,), (3, 4099)):
        v = values(rng, shape, f, dtype)
        want = oracle.quantize(v, f)
        q, lo, hi = c.quantize(dev(v), f)
        got = q.cpu().numpy()
        assert got.shape == v.shape
        assert np.array_equal(got, want), (shape, f)
        assert (lo, hi) == (int(want.min()), int(want.max()))


def test_quantize_errors_and_bounds():
    c = ccm()
    rng = np.random.default_rng(5)
    v = rng.standard_normal(5000)
    for pos in (0, 2500, 4999):
        for bad in (math.nan, math.inf, -math.inf):
            w = v.copy()
            w[pos] = bad
            w[(pos + 7) % 5000] = 2.0 ** 80  # an overflow elsewhere: NaN / inf decides
            with pytest.raises(c.CcmError) as e:
                c.quantize(dev(w), 3)
            assert e.value.status == c.E_RANGE
            with pytest.raises(c.CcmError) as e:
                c.float_absmax(dev(w))
            assert e.value.status == c.E_RANGE
    for f in (0, 10, -10):
        edge = math.ldexp(1.0, 62 - f)
        for x in (edge, -edge):
            w = v.copy()
            w[4321] = x
            with pytest.raises(c.CcmError) as e:
                c.quantize(dev(w), f)
            assert e.value.status == c.E_OVERFLOW
        below = math.nextafter(edge, 0.0)
        w = v.copy()
        w[17], w[18] = below, -below
        q, lo, hi = c.quantize(dev(w), f)
        assert (lo, hi) == (-(1 << 62) + 512, (1 << 62) - 512)
        assert np.array_equal(q.cpu().numpy(), oracle.quantize(w, f))
    # int32 output: the same q while it fits int32 (both ends exactly), an
    # overflow as soon as one q leaves it (2^31 - 1/2 rounds to the even 2^31)
    for f in (0, 5, -3):
        w = v.copy() * 1000.0
        w[10], w[11] = math.ldexp((1 << 31) - 1, -f), math.ldexp(-(1 << 31), -f)
        q, lo, hi = c.quantize(dev(w), f, dtype=torch.int32)
        assert q.dtype == torch.int32 and (lo, hi) == (-(1 << 31), (1 << 31) - 1)
        assert np.array_equal(q.cpu().numpy().astype(np.int64), oracle.quantize(w, f))
        for x in (math.ldexp((1 << 31) - 0.5, -f), math.ldexp(-(1 << 31) - 1.0, -f)):
            w2 = w.copy()
            w2[12] = x
            with pytest.raises(c.CcmError) as e:
                c.quantize(dev(w2), f, dtype=torch.int32)
            assert e.value.status == c.E_OVERFLOW
        w2 = w.copy()
        w2[12] = math.ldexp(-(1 << 31) - 0.5, -f)  # the tie rounds to the even -2^31
        q, lo, _ = c.quantize(dev(w2), f, dtype=torch.int32)
        assert lo == -(1 << 31)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_absmax_and_frac_bits(dtype):
    c = ccm()
    rng = np.random.default_rng(9)
    for n in (1, 100, 100000):
        for scale in (1e-30, 1.0, 1e30):
            v = (rng.standard_normal(n) * scale).astype(dtype)
            a = c.float_absmax(dev(v))
            assert a == float(np.abs(v.astype(np.float64)).max())
            for p in (1, 8, 24, 53):
                assert c.float_frac_bits(a, p) == oracle.frac_bits(a, p)
    assert c.float_absmax(dev(np.array([-0.0, 0.0], dtype=dtype))) == 0.0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_dequantize_matches_oracle(dtype):
    c = ccm()
    rng = np.random.default_rng(13)
    q = np.concatenate([rng.integers(-(1 << 62), 1 << 62, size=3000),
                        rng.integers(-(1 << 20), 1 << 20, size=3000),
                        [0, 1, -1, (1 << 53) + 1, -(1 << 53) - 3, (1 << 62) - 1,
                         -(1 << 62)]]).astype(np.int64)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    ut = np.uint32 if dtype == np.float32 else np.uint64
    for f in (0, 3, 40, -5, -60, 1074, 1100, 1200, 2400, -2400):
        got = c.dequantize(dev(q), f, tdt).cpu().numpy()
        want = oracle.dequantize(q, f, dtype)
        assert np.array_equal(got.view(ut), want.view(ut)), f


@pytest.mark.parametrize("f,shape", [(4, (5, 7)), (-2, (33, 65)), (20, (130, 1000)),
                                     (0, (1, 4099)), (60, (300, 301))])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_compress_float_matches_oracle(f, shape, dtype):
    """Header (fixed-point flag and scale) and payload bytes equal the
    oracle's encoding of its own quantization; decompress returns the
    oracle's dequantized matrix in both float types."""
    c = ccm()
    rng = np.random.default_rng(17 + f)
    v = values(rng, shape, f, dtype)
    m = c.compress_float(dev(v), frac_bits=f)
    p = oracle.compress(oracle.quantize(v, f))
    assert m.frac_bits == f and (m.bits, m.vmin, m.vmax) == (p.bits, p.vmin, p.vmax)
    assert m.header() == oracle.header_fx(p, f)
    assert m.payload_bytes() == p.payload_bytes()
    for odt, ut in ((torch.float64, np.uint64), (torch.float32, np.uint32)):
        got = c.decompress_float(m, odt).cpu().numpy()
        want = oracle.dequantize(oracle.decompress(p), f, np.float32 if ut == np.uint32
                                 else np.float64)
        assert np.array_equal(got.view(ut), want.view(ut))
    back = c.from_serialized(m.serialize())
    assert back.frac_bits == f and back.header() == m.header()
    assert torch.equal(c.decompress(back), c.decompress(m))


def test_significant_bits():
    """sig_bits p: f from the exact largest magnitude, the width of q within
    p .. p + 2 bits, and the rounding error within 2^-(f+1)."""
    c = ccm()
    rng = np.random.default_rng(21)
    for p in (1, 4, 8, 11, 16, 24, 40):
        v = rng.standard_normal(size=(64, 200)) * 10.0 ** int(rng.integers(-8, 8))
        m = c.compress_float(dev(v), sig_bits=p)
        f = oracle.frac_bits(float(np.abs(v).max()), p)
        assert m.frac_bits == f and p <= m.bits <= p + 2
        back = c.decompress_float(m).cpu().numpy()
        assert np.all(np.abs(back - v) <= math.ldexp(0.5, -f))


@pytest.mark.parametrize("shape", [(1, 1), (7, 130), (300, 4096), (1000, 16384 + 128)])
def test_matvec_float_matches_oracle(shape):
    """y = V x: x quantized, the exact integer matvec, y at f + g: every
    entry's bit pattern equals the oracle's."""
    c = ccm()
    rows, cols = shape
    rng = np.random.default_rng(rows + cols)
    v = values(rng, shape, 10)
    f = oracle.frac_bits(float(np.abs(v).max()), 12)
    x = rng.standard_normal(cols).astype(np.float32)
    g = oracle.frac_bits(float(np.abs(x.astype(np.float64)).max()), 16)
    m = c.compress_float(dev(v), frac_bits=f)
    y = c.matvec_float(m, dev(x), x_frac_bits=g).cpu().numpy()
    p = oracle.compress(oracle.quantize(v, f))
    want = oracle.dequantize(oracle.matvec(p, oracle.quantize(x, g)), f + g)
    assert np.array_equal(y.view(np.uint64), want.view(np.uint64))
    y2 = c.matvec_float(m, dev(x), x_sig_bits=16).cpu().numpy()
    assert np.array_equal(y2.view(np.uint64), want.view(np.uint64))
    # x kept to 14 significant bits: the int32 vector the fast matvec path takes
    g14 = oracle.frac_bits(float(np.abs(x.astype(np.float64)).max()), 14)
    y3 = c.matvec_float(m, dev(x), x_sig_bits=14).cpu().numpy()
    want3 = oracle.dequantize(oracle.matvec(p, oracle.quantize(x, g14)), f + g14)
    assert np.array_equal(y3.view(np.uint64), want3.view(np.uint64))


def test_matvec_float_overflow_rule():
    c = ccm()
    v = np.full((4, 1000), 2.0 ** 30)
    m = c.compress_float(dev(v), frac_bits=0)
    with pytest.raises(c.CcmError) as e:
        c.matvec_float(m, dev(np.full(1000, 2.0 ** 24)), x_frac_bits=0)
    assert e.value.status == c.E_OVERFLOW
    y = c.matvec_float(m, dev(np.full(1000, 2.0 ** 22)), x_frac_bits=0).cpu().numpy()
    assert np.all(y == 1000 * 2.0 ** 52)


def test_scale_carried_through_operations():
    """add (same scale only), scale by an integer, matmul (scales add) and
    the transpose keep the fixed-point scale; results equal the oracle's
    exact integer results on q."""
    c = ccm()
    rng = np.random.default_rng(25)
    a = values(rng, (40, 70), 6)
    b = values(rng, (40, 70), 6)
    qa, qb = oracle.quantize(a, 6), oracle.quantize(b, 6)
    ma, mb = c.compress_float(dev(a), frac_bits=6), c.compress_float(dev(b), frac_bits=6)
    s = c.add(ma, mb)
    assert s.frac_bits == 6
    want = oracle.dequantize(oracle.decompress(oracle.add(oracle.compress(qa),
                                                          oracle.compress(qb))), 6)
    assert np.array_equal(c.decompress_float(s).cpu().numpy(), want)
    with pytest.raises(c.CcmError):
        c.add(ma, c.compress_float(dev(b), frac_bits=7))
    t = c.scale(ma, -3)
    assert t.frac_bits == 6
    assert np.array_equal(c.decompress_float(t).cpu().numpy(),
                          oracle.dequantize(-3 * qa, 6))
    small = np.ldexp(rng.integers(-60, 60, size=(70, 30)).astype(np.float64), -2)
    mm = c.matmul(ma, c.compress_float(dev(small), frac_bits=2))
    assert mm.frac_bits == 8
    qs = oracle.quantize(small, 2)
    want = oracle.dequantize(oracle.decompress(oracle.matmul(oracle.compress(qa),
                                                             oracle.compress(qs))), 8)
    assert np.array_equal(c.decompress_float(mm).cpu().numpy(), want)
    assert ma.T.frac_bits == 6


def test_float_workload_full_size_sampled():
    """The benchmark's 16384^2 float32 matrix at 12 significant bits, built
    on the device as the benchmark builds it: the fraction bits from the
    exact largest magnitude and the header from the exact range of q, both
    computed on the host over all 2^28 elements; sampled rows of the payload,
    of decompress_float and of matvec_float equal the oracle's."""
    c = ccm()
    n = 16384
    ms, es, xs = W.float_matrix(n)
    mt = torch.empty((n, n), dtype=torch.int32, device="cuda")
    et = torch.empty((n, n), dtype=torch.int32, device="cuda")
    c.fill_uniform(mt, ms.lo, ms.hi, ms.seed, ms.stream)
    c.fill_uniform(et, es.lo, es.hi, es.seed, es.stream)
    V = torch.ldexp(mt.to(torch.float32), et.to(torch.float32))
    del mt, et
    xm = torch.empty(n, dtype=torch.int32, device="cuda")
    c.fill_uniform(xm, xs.lo, xs.hi, xs.seed, xs.stream)
    x = torch.ldexp(xm.to(torch.float32), torch.full((n,), -23.0, device="cuda"))
    m = c.compress_float(V, sig_bits=12)
    y = c.matvec_float(m, x, x_sig_bits=14).cpu().numpy()
    back = c.decompress_float(m, torch.float32)
    torch.cuda.synchronize()

    def rows_of(r0, r1):
        return np.ldexp(ms.rows_slice(r0, r1).astype(np.float64),
                        es.rows_slice(r0, r1)).astype(np.float32)

    def amax(r0):
        return float(np.abs(rows_of(r0, min(n, r0 + 1024)).astype(np.float64)).max())
    with ThreadPoolExecutor(8) as ex:
        a = max(ex.map(amax, range(0, n, 1024)))
    f = oracle.frac_bits(a, 12)
    assert m.frac_bits == f

    def qrange(r0):
        q = oracle.quantize(rows_of(r0, min(n, r0 + 1024)), f)
        return int(q.min()), int(q.max())
    with ThreadPoolExecutor(8) as ex:
        parts = list(ex.map(qrange, range(0, n, 1024)))
    lo, hi = min(p[0] for p in parts), max(p[1] for p in parts)
    assert m.header() == oracle.header_fx_of(n, n, lo, hi, f)
    bits, sgn = oracle.width(lo, hi)
    xv = np.ldexp(xs.dense().astype(np.float64), -23).astype(np.float32)
    g = oracle.frac_bits(float(np.abs(xv.astype(np.float64)).max()), 14)
    xq = oracle.quantize(xv, g)
    per_row = n * bits // 64
    for r in (0, 1, 4095, 8192, 12345, n - 1):
        q = oracle.quantize(rows_of(r, r + 1), f)
        words = oracle.encode_run(q, bits)
        got = np.frombuffer(m.payload[8 * r * per_row: 8 * (r + 1) * per_row].cpu().numpy()
                            .tobytes(), dtype="<u8")
        assert np.array_equal(got, words[: per_row])
        assert np.array_equal(back[r].cpu().numpy().view(np.uint32),
                              oracle.dequantize(q[0], f, np.float32).view(np.uint32))
        p = oracle.Packed(1, n, int(q.min()), int(q.max()), bits, sgn, words)
        want = oracle.dequantize(oracle.matvec(p, xq), f + g)
        assert y[r:r + 1].view(np.uint64).tolist() == want.view(np.uint64).tolist()
