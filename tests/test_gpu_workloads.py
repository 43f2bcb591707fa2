"""Workload-sized parity checks (GPU vs oracle) in the configurations the
benchmark times.  The oracle cannot process whole 2^28-element matrices, so
it checks sampled rows (the encoding is local: a row that starts on a 64-bit
boundary encodes to its own bitstrings) and sampled entries; headers are
checked exactly where the full value range can be computed on the host."""
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


def full_range(spec, chunk_rows=2048):
    lo, hi = None, None
    for r in range(0, spec.rows, chunk_rows):
        v = spec.rows_slice(r, min(spec.rows, r + chunk_rows))
        lo = int(v.min()) if lo is None else min(lo, int(v.min()))
        hi = int(v.max()) if hi is None else max(hi, int(v.max()))
    return lo, hi


@pytest.mark.parametrize("k", list(W.SWEEP_WIDTHS))
@pytest.mark.parametrize("signed", [False, True])
def test_sweep_full_size_sampled(k, signed):
    c = ccm()
    a_s, b_s, x_s, s = W.sweep(k, signed, N_SWEEP)
    dense = torch.empty((N_SWEEP, N_SWEEP), dtype=torch.int64, device="cuda")
    c.fill_uniform(dense, a_s.lo, a_s.hi, a_s.seed, a_s.stream)
    A = c.compress(dense)
    c.fill_uniform(dense, b_s.lo, b_s.hi, b_s.seed, b_s.stream)
    B = c.compress(dense)
    del dense
    assert (A.bits, A.is_signed) == (k, signed)
    assert a_s.lo <= A.vmin and A.vmax <= a_s.hi - 1
    if (k, signed) in ((3, False), (31, True)):
        assert (A.vmin, A.vmax) == full_range(a_s)
    x = torch.empty(N_SWEEP, dtype=torch.int32, device="cuda")
    c.fill_uniform(x, x_s.lo, x_s.hi, x_s.seed, x_s.stream)
    y = c.matvec(A, x).cpu().numpy()
    xv = x_s.dense()
    sum_ = c.add(A, B)
    scaled = c.scale(A, s)
    for r in SAMPLE_ROWS:
        va, pa = oracle_rows(a_s, [r], A.bits, A.is_signed)
        vb, pb = oracle_rows(b_s, [r], B.bits, B.is_signed)
        # compress: the row's bitstrings
        assert np.array_equal(words_of_rows(A, r, r + 1), pa.payload[: pa.words - 1])
        # matvec
        assert y[r] == oracle.matvec(pa, xv)[0]
        # add and scale, re-encoded at the GPU result's width
        want = oracle.encode_run(oracle.add_dense(pa, pb), sum_.bits)
        assert np.array_equal(words_of_rows(sum_, r, r + 1), want[: len(want) - 1])
        want = oracle.encode_run(oracle.scale_dense(pa, s), scaled.bits)
        assert np.array_equal(words_of_rows(scaled, r, r + 1), want[: len(want) - 1])
    # result widths follow from the operand ranges
    assert sum_.bits == oracle.width(A.vmin + B.vmin, A.vmax + B.vmax)[0] or \
        sum_.bits == oracle.width(sum_.vmin, sum_.vmax)[0]
    assert (scaled.vmin, scaled.vmax) == (min(s * A.vmin, s * A.vmax), max(s * A.vmin, s * A.vmax))


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
    assert (C.vmin, C.vmax) == (lo, hi)
    assert (C.bits, C.is_signed) == oracle.width(lo, hi)
    # a few full rows of C, bit for bit
    for r in (0, 4097, 8191):
        row = exact[r].astype(np.int64)
        per_row = 8192 * C.bits // 64
        got_w = np.frombuffer(C.payload[8 * r * per_row: 8 * (r + 1) * per_row].cpu().numpy()
                              .tobytes(), dtype="<u8")
        assert np.array_equal(got_w.astype(np.uint64),
                              oracle.encode_run(row, C.bits)[: per_row])
