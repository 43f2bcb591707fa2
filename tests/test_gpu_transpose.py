"""Column-major unravel and y = A^T x on the GPU against the CPU oracle.

A column-major matrix's payload and header are compared byte for byte with
the oracle's column-major encoding; decompress, get, gather, add and scale
keep the order; y = A x and y = A^T x are compared element by element for
both orders, through both packing kernels (rows a multiple of 32 or not) and
with rows split over several blocks.  The full-size case checks the identity
z . (A^T x) = x . (A z) modulo 2^64 between the two matvec kernels.
"""
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


def dev(a, dtype=torch.int64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def rand_matrix(rng, rows, cols, b, signed):
    lo, hi = ((-(1 << (b - 1)), (1 << (b - 1)) - 1) if signed else (0, (1 << b) - 1))
    m = rng.integers(lo, hi, size=(rows, cols), endpoint=True, dtype=np.int64)
    flat = m.reshape(-1)
    flat[int(rng.integers(0, flat.size))] = hi
    if signed:
        flat[int(rng.integers(0, flat.size))] = lo
    return m


def payload_words(g):
    torch.cuda.synchronize()
    return g.payload[: 8 * g.words].cpu().numpy().view(np.uint64)


def check_cm(g, ref, A, rng):
    c = ccm()
    assert g.order == "F" and g.shape == A.shape
    assert g.header() == oracle.header_cm(ref)
    assert np.array_equal(payload_words(g), ref.payload)
    assert not g.payload[8 * g.words:].cpu().numpy().any()
    assert np.array_equal(c.decompress(g).cpu().numpy(), A)
    rows, cols = A.shape
    for i, j in [(0, 0), (rows - 1, cols - 1), (int(rng.integers(0, rows)), int(rng.integers(0, cols)))]:
        assert c.get(g, i, j) == int(A[i, j]) == oracle.get_cm(ref, i, j)


def narrow_x(rng, n, wide_at=None):
    """x in [-2^15, 2^15) with both ends present; optionally one value past it."""
    x = rng.integers(-(1 << 15), (1 << 15) - 1, size=n, endpoint=True, dtype=np.int64)
    x[int(rng.integers(0, n))] = -(1 << 15)
    x[int(rng.integers(0, n))] = (1 << 15) - 1
    if wide_at is not None:
        x[wide_at] = 1 << 15
    return x


def check_products(g, A, rng):
    """matvec and matvec_t of g (either order) against the oracle: x over the
    whole int32 and int64 ranges, x in [-2^15, 2^15) (the 32-bit partial sums
    of y = A^T x), and such x with one value just past that range."""
    c = ccm()
    rows, cols = A.shape
    pr = oracle.compress(A)
    for xdt, lo, hi in [(torch.int32, -(1 << 31), (1 << 31) - 1), (torch.int64, -2**62, 2**62)]:
        xc = rng.integers(lo, hi, size=cols, endpoint=True, dtype=np.int64)
        xr = rng.integers(lo, hi, size=rows, endpoint=True, dtype=np.int64)
        assert np.array_equal(c.matvec(g, dev(xc, xdt)).cpu().numpy(), oracle.matvec(pr, xc))
        assert np.array_equal(c.matvec_t(g, dev(xr, xdt)).cpu().numpy(), oracle.matvec_t(pr, xr))
    for xdt in (torch.int32, torch.int64):
        for wide_at in (None, int(rng.integers(0, rows))):
            xr = narrow_x(rng, rows, wide_at)
            assert np.array_equal(c.matvec_t(g, dev(xr, xdt)).cpu().numpy(),
                                  oracle.matvec_t(pr, xr))


SHAPES = [(1, 1), (1, 40), (40, 1), (32, 7), (64, 100), (37, 33), (96, 2100), (130, 257),
          (2049, 3), (300, 4200)]


@pytest.mark.parametrize("b", list(range(1, 65)))
def test_column_major_all_widths(b):
    c = ccm()
    rng = np.random.default_rng(500 + b)
    for signed in ((False, True) if b < 64 else (True,)):
        for rows, cols in SHAPES[: 4 + b % 7]:
            if signed and b == 1 and rows * cols < 2:
                continue
            A = rand_matrix(rng, rows, cols, b, signed)
            ref = oracle.compress_cm(A)
            g = c.compress(dev(A), order="F")
            check_cm(g, ref, A, rng)
            if b <= 31:
                check_cm(c.compress(dev(A, torch.int32), order="F"), ref, A, rng)
            check_products(g, A, rng)
            # the row-major matrix: y = A^T x through the transposed kernel
            check_products(c.compress(dev(A)), A, rng)


@pytest.mark.parametrize("shape", [(5000, 70), (4096, 4096), (777, 5000)], ids=str)
@pytest.mark.parametrize("b", [1, 3, 12, 31, 40])
def test_transposed_split_rows(shape, b):
    """Rows split over several blocks (atomic column sums), several panels."""
    c = ccm()
    rng = np.random.default_rng(b * 7 + shape[0])
    A = rand_matrix(rng, *shape, b, b % 2 == 1)
    check_products(c.compress(dev(A)), A, rng)


@pytest.mark.parametrize("b", [1, 3, 7, 8, 9, 12, 13, 14, 15])
def test_transposed_narrow_extremes(b):
    """The 32-bit partial sums at their bound: every field at its largest
    magnitude and every x at -2^15 (then 2^15 - 1), with enough rows per wave
    that the wider fields fold their partial sums several times."""
    c = ccm()
    rows, cols = 40000, 64
    for signed in (False, True):
        a = -(1 << (b - 1)) if signed else (1 << b) - 1
        A = np.full((rows, cols), a, dtype=np.int64)
        A[0, 0] = 0 if not signed else (1 << (b - 1)) - 1  # keep the width at b
        g = c.compress(dev(A))
        assert g.bits == b and g.is_signed == signed
        pr = oracle.compress(A)
        for xv in (-(1 << 15), (1 << 15) - 1):
            x = np.full(rows, xv, dtype=np.int64)
            assert np.array_equal(c.matvec_t(g, dev(x, torch.int32)).cpu().numpy(),
                                  oracle.matvec_t(pr, x)), (signed, xv)


@pytest.mark.parametrize("b", [7, 8])
def test_transposed_long_waves(b):
    """Rows per wave past the 32-bit run length (b <= 8 takes 64-bit products
    then, whatever x)."""
    c = ccm()
    rng = np.random.default_rng(40 + b)
    A = rand_matrix(rng, 300000, 40, b, False)
    g = c.compress(dev(A))
    pr = oracle.compress(A)
    x = narrow_x(rng, A.shape[0])
    assert np.array_equal(c.matvec_t(g, dev(x, torch.int32)).cpu().numpy(), oracle.matvec_t(pr, x))


@pytest.mark.parametrize("shape", [(5000, 70), (4096, 4096), (777, 5000)], ids=str)
def test_transposed_without_scratch(shape):
    """ccm_matvec_t with scratch NULL (row splits added with atomics) and with
    one scratch buffer reused by consecutive calls, against the oracle."""
    import ctypes
    c = ccm()
    rng = np.random.default_rng(shape[1])
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    nb = None
    scratch = None
    for b in (1, 12, 40):
        A = rand_matrix(rng, *shape, b, True)
        g = c.compress(dev(A))
        pr = oracle.compress(A)
        if scratch is None:
            nb = int(c.lib.ccm_matvec_t_scratch_bytes(ctypes.byref(g.desc)))
            assert nb == 8 * 32 * shape[1]
            scratch = torch.empty(nb // 8, dtype=torch.int64, device="cuda")
        for xr in (narrow_x(rng, shape[0]),
                   rng.integers(-(1 << 31), (1 << 31) - 1, size=shape[0], dtype=np.int64)):
            x = dev(xr, torch.int32)
            want = oracle.matvec_t(pr, xr)
            for sp, sb in ((None, 0), (ctypes.c_void_p(scratch.data_ptr()), nb)):
                y = torch.full((shape[1],), 7, dtype=torch.int64, device="cuda")
                rc = c.lib.ccm_matvec_t(ctypes.byref(g.desc), ctypes.c_void_p(x.data_ptr()),
                                        c.I32, ctypes.c_void_p(y.data_ptr()), sp, sb, s)
                assert rc == 0
                assert np.array_equal(y.cpu().numpy(), want), (b, sp is None)


def test_transpose_view_and_ops():
    c = ccm()
    rng = np.random.default_rng(9)
    A = rand_matrix(rng, 70, 45, 9, True)
    B = rand_matrix(rng, 70, 45, 5, False)
    gA = c.compress(dev(A))
    t = gA.T  # the transpose, same payload, column-major
    assert t.order == "F" and t.shape == (45, 70)
    assert np.array_equal(c.decompress(t).cpu().numpy(), A.T)
    assert c.get(t, 3, 60) == int(A[60, 3])
    assert t.T.order == "C" and np.array_equal(c.decompress(t.T).cpu().numpy(), A)
    check_products(t, A.T, rng)
    fA, fB = c.compress(dev(A), order="F"), c.compress(dev(B), order="F")
    s = c.add(fA, fB)
    assert s.order == "F" and np.array_equal(c.decompress(s).cpu().numpy(), A + B)
    k = c.scale(fA, -3)
    assert k.order == "F" and np.array_equal(c.decompress(k).cpu().numpy(), -3 * A)
    ii = torch.tensor([0, 69, 5], device="cuda")
    jj = torch.tensor([0, 44, 40], device="cuda")
    vals, bad = c.gather(fA, ii, jj)
    assert vals.cpu().tolist() == [int(A[0, 0]), int(A[69, 44]), int(A[5, 40])] and not bad
    blob = fA.serialize()
    assert blob[7] & 2 and blob[:64] == oracle.header_cm(oracle.compress_cm(A))
    back = c.from_serialized(blob)
    assert back.order == "F" and np.array_equal(c.decompress(back).cpu().numpy(), A)
    with pytest.raises(c.CcmError):
        c.add(gA, fB)
    with pytest.raises(c.CcmError):
        c.matmul(fA, c.compress(dev(B.T)))
    with pytest.raises(c.CcmError):
        c.matvec_t(gA, torch.zeros(45, dtype=torch.int32, device="cuda"))


def test_worked_example_column():
    """The paper's example row as a column: the same two bitstrings."""
    c = ccm()
    vals = np.array([[900, 1023, 721, 256, 1, 10, 700, 20]])
    g = c.compress(dev(vals.T), order="F")
    assert np.array_equal(payload_words(g), oracle.compress(vals).payload)
    assert c.decompress(g).cpu().numpy().tolist() == vals.T.tolist()


@pytest.mark.parametrize("k", [3, 12, 31])
def test_full_size_identity(k):
    """16384 x 16384 sweep matrix: z . (A^T x) == x . (A z) modulo 2^64, the
    two sides from the two matvec kernels."""
    c = ccm()
    a_s, _, _, _ = W.sweep(k, False)
    A = c.generate(a_s.rows, a_s.cols, a_s.lo, a_s.hi, a_s.seed, a_s.stream)
    rng = np.random.default_rng(k)
    x = rng.integers(-(1 << 15), 1 << 15, size=a_s.rows, dtype=np.int64)
    z = rng.integers(-(1 << 15), 1 << 15, size=a_s.cols, dtype=np.int64)
    aty = c.matvec_t(A, dev(x, torch.int32)).cpu().numpy()
    az = c.matvec(A, dev(z, torch.int32)).cpu().numpy()
    m = (1 << 64) - 1
    lhs = sum(int(u) * int(v) for u, v in zip(z, aty)) & m
    rhs = sum(int(u) * int(v) for u, v in zip(x, az)) & m
    assert lhs == rhs


@pytest.mark.parametrize("k,signed", [(1, False), (12, True), (31, False)])
def test_full_size_sampled_columns(k, signed):
    """y = A^T x on the 16384 x 16384 sweep matrix with the sweep's x, launched
    as the benchmark launches it (pre-marshalled, scratch for the row splits):
    sampled columns against the oracle's A^T x of that column alone, the
    column regenerated on the host."""
    c = ccm()
    a_s, _, x_s, _ = W.sweep(k, signed)
    A = c.generate(a_s.rows, a_s.cols, a_s.lo, a_s.hi, a_s.seed, a_s.stream)
    x = torch.empty(a_s.rows, dtype=torch.int32, device="cuda")
    c.fill_uniform(x, x_s.lo, x_s.hi, x_s.seed, x_s.stream)
    y = torch.full((a_s.cols,), 5, dtype=torch.int64, device="cuda")
    go = c.matvec_launcher(A, x, y, transposed=True)
    go()
    go()  # a second call reuses the scratch
    got = y.cpu().numpy()
    xh = x_s.dense()
    assert np.array_equal(x.cpu().numpy(), xh)
    rng = np.random.default_rng(k)
    cols = sorted({0, 1, 31, 32, 2047, 2048, a_s.cols - 1} |
                  {int(j) for j in rng.integers(0, a_s.cols, 5)})
    for j in cols:
        col = a_s.column(j).reshape(-1, 1)
        want = oracle.matvec_t(oracle.compress(col), xh)
        assert got[j] == want[0], j

