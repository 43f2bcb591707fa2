"""Workload-sized parity checks (GPU vs oracle) in the configurations the
benchmark times.  The oracle cannot process whole 2^28-element matrices, so
it checks sampled rows (the encoding is local: a row that starts on a 64-bit
boundary encodes to its own bitstrings) and sampled entries; headers are
checked exactly where the full value range can be computed on the host."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import ccm_workloads as W
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_SWEEP = 16384
SAMPLE_ROWS = [0, 1, 2, 1000, 8191, 8192, 12345, N_SWEEP - 1]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "gpu tests need a GPU"


def ccm():
    import paper_1303_0270_amd as c
    return c


def words_of_rows(m, r0, r1):
    """Payload 64-bit words of rows [r0, r1) (rows start on 64-bit boundaries)."""
    per_row = m.cols * m.bits // 64
    lo, hi = r0 * per_row, r1 * per_row
    return np.frombuffer(
        m.payload[8 * lo: 8 * hi].cpu().numpy().tobytes(), dtype="<u8").astype(np.uint64)


def oracle_rows(spec, rows, bits, signed):
    vals = np.concatenate([spec.rows_slice(r, r + 1) for r in rows])
    return vals, oracle.Packed(len(rows), spec.cols, int(vals.min()), int(vals.max()), bits,
                               signed, oracle.encode_run(vals, bits))


def exact_ranges(a_s, b_s, chunk_rows=1024, workers=8):
    """Exact extremes of A, of B and of A + B over the whole matrices, drawn
    again on the host from the seeded generator, in row chunks."""
    def part(r0):
        r1 = min(a_s.rows, r0 + chunk_rows)
        va, vb = a_s.rows_slice(r0, r1), b_s.rows_slice(r0, r1)
        sm = va + vb
        return (int(va.min()), int(va.max()), int(vb.min()), int(vb.max()),
                int(sm.min()), int(sm.max()))
    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(part, range(0, a_s.rows, chunk_rows)))
    lo = lambda i: min(p[i] for p in parts)
    hi = lambda i: max(p[i] for p in parts)
    return (lo(0), hi(1)), (lo(2), hi(3)), (lo(4), hi(5))


@pytest.mark.parametrize("k", list(W.SWEEP_WIDTHS))
@pytest.mark.parametrize("signed", [False, True])
def test_sweep_full_size_sampled(k, signed):
    """The full 16384^2 sweep case as the benchmark runs it.  Every result's
    header (width, signedness, exact extremes, bitstring count) equals the
    oracle's header for the exact range of its values, computed on the host
    over all 2^28 elements; sampled rows of every payload equal the oracle's
    encoding at the oracle's width; sampled rows of matvec and decompress
    equal the oracle's."""
    c = ccm()
    a_s, b_s, x_s, s = W.sweep(k, signed, N_SWEEP)
    dense = torch.empty((N_SWEEP, N_SWEEP), dtype=torch.int64, device="cuda")
    c.fill_uniform(dense, a_s.lo, a_s.hi, a_s.seed, a_s.stream)
    A = c.compress(dense)
    c.fill_uniform(dense, b_s.lo, b_s.hi, b_s.seed, b_s.stream)
    B = c.compress(dense)
    x = torch.empty(N_SWEEP, dtype=torch.int32, device="cuda")
    c.fill_uniform(x, x_s.lo, x_s.hi, x_s.seed, x_s.stream)
    y = c.matvec(A, x).cpu().numpy()
    sum_ = c.add(A, B)
    scaled = c.scale(A, s)
    dec = c.decompress(A, out=dense)
    torch.cuda.synchronize()

    ra, rb, rs = exact_ranges(a_s, b_s)
    rsc = (min(s * ra[0], s * ra[1]), max(s * ra[0], s * ra[1]))
    assert A.header() == oracle.header_of(N_SWEEP, N_SWEEP, *ra)
    assert B.header() == oracle.header_of(N_SWEEP, N_SWEEP, *rb)
    assert sum_.header() == oracle.header_of(N_SWEEP, N_SWEEP, *rs)
    assert scaled.header() == oracle.header_of(N_SWEEP, N_SWEEP, *rsc)
    (abits, asgn), (bbits, bsgn) = oracle.width(*ra), oracle.width(*rb)
    sbits, cbits = oracle.width(*rs)[0], oracle.width(*rsc)[0]
    assert (abits, asgn) == (k, signed)

    xv = x_s.dense()
    for r in SAMPLE_ROWS:
        va, pa = oracle_rows(a_s, [r], abits, asgn)
        vb, pb = oracle_rows(b_s, [r], bbits, bsgn)
        # compress: the row's bitstrings
        assert np.array_equal(words_of_rows(A, r, r + 1), pa.payload[: pa.words - 1])
        # decompress: the row's values, as the oracle decodes them
        got = dec[r].cpu().numpy()
        assert np.array_equal(got, oracle.decompress(pa)[0]) and np.array_equal(got, va[0])
        # matvec
        assert y[r] == oracle.matvec(pa, xv)[0]
        # add and scale, encoded at the oracle's width of the exact result range
        want = oracle.encode_run(oracle.add_dense(pa, pb), sbits)
        assert np.array_equal(words_of_rows(sum_, r, r + 1), want[: len(want) - 1])
        want = oracle.encode_run(oracle.scale_dense(pa, s), cbits)
        assert np.array_equal(words_of_rows(scaled, r, r + 1), want[: len(want) - 1])


def test_dense_gemm_full_size_sampled():
    """8192^3, A in [0, 2^6), B in [-2^3, 2^3): sampled entries against the
    oracle, and C's exact range from a float64 product (exact: |C| < 2^23)."""
    c = ccm()
    a_s, b_s = W.dense_gemm(8192)
    A = c.generate(a_s.rows, a_s.cols, a_s.lo, a_s.hi, a_s.seed, a_s.stream)
    B = c.generate(b_s.rows, b_s.cols, b_s.lo, b_s.hi, b_s.seed, b_s.stream)
    assert (A.bits, A.is_signed, B.bits, B.is_signed) == (6, False, 4, True)
    C = c.matmul(A, B)
    Ad, Bd = a_s.dense(), b_s.dense()
    pa = oracle.Packed(8192, 8192, int(Ad.min()), int(Ad.max()), 6, False,
                       oracle.encode_run(Ad, 6))
    pb = oracle.Packed(8192, 8192, int(Bd.min()), int(Bd.max()), 4, True,
                       oracle.encode_run(Bd, 4))
    rng = np.random.default_rng(W.seed_for(3, 3))
    ii = np.concatenate([[0, 0, 8191, 8191, 127, 128], rng.integers(0, 8192, 250)])
    jj = np.concatenate([[0, 8191, 0, 8191, 128, 127], rng.integers(0, 8192, 250)])
    want = oracle.matmul_entries(pa, pb, ii, jj)
    got, bad = c.gather(C, torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda())
    assert not bad
    assert np.array_equal(got.cpu().numpy(), want)
    exact = (Ad.astype(np.float64) @ Bd.astype(np.float64))
    lo, hi = int(exact.min()), int(exact.max())
    assert C.header() == oracle.header_of(8192, 8192, lo, hi)
    cbits = oracle.width(lo, hi)[0]
    # a few full rows of C, bit for bit, at the oracle's width
    for r in (0, 4097, 8191):
        row = exact[r].astype(np.int64)
        per_row = 8192 * cbits // 64
        got_w = np.frombuffer(C.payload[8 * r * per_row: 8 * (r + 1) * per_row].cpu().numpy()
                              .tobytes(), dtype="<u8")
        assert np.array_equal(got_w.astype(np.uint64),
                              oracle.encode_run(row, cbits)[: per_row])
