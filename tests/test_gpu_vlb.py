"""Method 2 (variable length blocks) on the GPU against the CPU oracle.

Bit-exact: the canonical payload words, the index (row starts and group
offsets, checked against the oracle's element start bits), decompress, get and
matvec.  Shapes cover one and several staged panels, ragged row ends, partial
panels, both matvec kernels (staged for aligned int32 x, general for int64 or
unaligned x), widths past 32 bits, signed matrices and the degenerate cases.
"""
import zlib

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


def check_encoding(g, ref):
    """GPU stream and index against the oracle."""
    assert (g.rows, g.cols, g.vmin, g.vmax) == (ref.rows, ref.cols, ref.vmin, ref.vmax)
    assert (g.k, g.is_signed, g.nbits, g.words) == (ref.k, ref.is_signed, ref.nbits, ref.words)
    got = g.payload_words().numpy().view(np.uint64)
    assert np.array_equal(got, ref.payload)
    # the whole capacity past the canonical payload is zero
    assert not g.payload[8 * g.words:].cpu().numpy().any()
    starts = oracle.vlb_offsets(ref, 32).astype(np.int64)
    rb = g.row_bits().numpy()
    assert rb[0] == 0 and rb[-1] == ref.nbits
    assert np.array_equal(rb[:-1], starts[:, 0])
    assert np.array_equal(g.group_offsets().numpy(), starts - starts[:, :1])
    ends = np.append(starts.ravel()[1:], ref.nbits)
    assert g.gmax == int((ends - starts.ravel()).max())


def check_ops(g, ref, A, rng, x_lo=-(1 << 31), x_hi=(1 << 31) - 1):
    c = ccm()
    assert np.array_equal(c.vlb_decompress(g).cpu().numpy(), A)
    rows, cols = A.shape
    picks = [(0, 0), (rows - 1, cols - 1)] + [
        (int(rng.integers(0, rows)), int(rng.integers(0, cols))) for _ in range(6)]
    for i, j in picks:
        assert c.vlb_get(g, i, j) == int(A[i, j]) == oracle.vlb_get(ref, i, j)
    x = rng.integers(x_lo, x_hi, size=cols, endpoint=True, dtype=np.int64)
    want = oracle.vlb_matvec(ref, x)
    # staged kernel: aligned int32 x
    x32 = dev(x, torch.int32)
    assert np.array_equal(c.vlb_matvec(g, x32).cpu().numpy(), want)
    # general kernel: int64 x, and int32 x off a 16-byte boundary
    assert np.array_equal(c.vlb_matvec(g, dev(x)).cpu().numpy(), want)
    buf = torch.empty(cols + 1, dtype=torch.int32, device="cuda")
    buf[1:] = x32
    assert np.array_equal(c.vlb_matvec(g, buf[1:]).cpu().numpy(), want)


def beta_matrix(rng, rows, cols, a1, b1, signed=False, max_len=63):
    """Bit-lengths from Beta(a1, b1) on [1, 64] (capped), values of exactly
    that length; signed: random signs."""
    x = rng.beta(a1, b1, size=rows * cols)
    L = np.minimum(np.floor(64 * x).astype(np.int64) + 1, max_len)
    top = np.left_shift(np.ones_like(L), L - 1)
    low = rng.integers(0, 1 << 62, size=L.size, dtype=np.int64)
    v = np.where(L == 1, low & 1, top | (low & (top - 1)))
    if signed:
        neg = rng.random(L.size) < 0.5
        v = np.where(neg, -v - 1, v)
    return v.reshape(rows, cols)


def test_worked_example_on_gpu():
    c = ccm()
    vals = np.array([[900, 1023, 721, 256, 1, 10, 700, 20]])
    ref = oracle.vlb_compress(vals)
    g = c.vlb_compress(dev(vals))
    check_encoding(g, ref)
    assert g.nbits == 91 and g.k == 4
    check_ops(g, ref, vals, np.random.default_rng(1))


SHAPES = [(1, 1), (1, 33), (3, 37), (65, 33), (130, 257), (7, 1000), (2, 16384), (3, 16416),
          (2, 32768 + 7), (9, 40000)]
DISTS = [("beta_1_32", 1.0, 32.0, False), ("beta_5_33", 5.0, 33.0, False),
         ("beta_1_1", 1.0, 1.0, False), ("beta_5_33_signed", 5.0, 33.0, True),
         ("beta_1_1_signed", 1.0, 1.0, True)]


@pytest.mark.parametrize("dist", DISTS, ids=lambda d: d[0])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
def test_parity(dist, shape):
    c = ccm()
    name, a1, b1, signed = dist
    rng = np.random.default_rng(zlib.crc32(repr((name, shape)).encode()))
    A = beta_matrix(rng, *shape, a1, b1, signed)
    ref = oracle.vlb_compress(A)
    g = c.vlb_compress(dev(A))
    check_encoding(g, ref)
    check_ops(g, ref, A, rng)


@pytest.mark.parametrize("top", [1, 2, 7, 25, 26, 27, 31, 32, 33, 57, 58, 63])
def test_width_boundaries(top):
    """Every element near one width: pairs just inside and just past the 32
    bits the staged kernel reads in one go (k + b = 32, 33), and the widest."""
    c = ccm()
    rng = np.random.default_rng(top)
    A = rng.integers(0, (1 << top) - 1, size=(5, 300), dtype=np.int64, endpoint=True)
    A |= 1 << (top - 1)
    A[0, 0] = 0
    for signed in (False, True):
        M = A if not signed else np.where(rng.random(A.shape) < 0.5, -A - 1, A)
        ref = oracle.vlb_compress(M)
        g = c.vlb_compress(dev(M))
        check_encoding(g, ref)
        check_ops(g, ref, M, rng)


def test_degenerate():
    c = ccm()
    rng = np.random.default_rng(5)
    cases = [np.zeros((4, 70), dtype=np.int64), np.ones((3, 3), dtype=np.int64),
             np.full((2, 5), -1, dtype=np.int64),
             np.array([[-2**63, 2**63 - 1, 0, -1, 1]], dtype=np.int64),
             np.full((1, 40000), 2**63 - 1, dtype=np.int64)]
    for A in cases:
        ref = oracle.vlb_compress(A)
        g = c.vlb_compress(dev(A))
        check_encoding(g, ref)
        check_ops(g, ref, A, rng)
    # int32 input encodes the same
    A = beta_matrix(rng, 33, 129, 5.0, 33.0, max_len=31)
    ref = oracle.vlb_compress(A)
    check_encoding(c.vlb_compress(dev(A, torch.int32)), ref)


def test_errors():
    c = ccm()
    g = c.vlb_compress(dev(np.arange(12).reshape(3, 4)))
    with pytest.raises(c.CcmError) as e:
        c.vlb_get(g, 3, 0)
    assert e.value.status == -3
    with pytest.raises(c.CcmError):
        c.vlb_matvec(g, torch.zeros(5, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("name", ["beta_5_33", "beta_1_1"])
def test_workload_full_size_sampled(name):
    """A 16384 x 16384 Beta matrix as the benchmark builds it (on the GPU):
    sampled rows' values, start bits and matvec outputs against the oracle
    run on those rows alone.  Beta(1, 1)'s stream is 10.3 G bits, so row
    starts and staged stretches lie past 2^32 bits."""
    c = ccm()
    spec, xs = W.vlb_sweep(name)
    A = spec.dense_device(c.fill_uniform, torch)
    g = c.vlb_compress(A)
    del A
    x = xs.dense()
    y = c.vlb_matvec(g, dev(x, torch.int32)).cpu().numpy()
    rb = g.row_bits().numpy()
    rng = np.random.default_rng(7)
    rows = sorted(set([0, spec.rows - 1] + [int(r) for r in rng.integers(0, spec.rows, 6)]))
    for r in rows:
        row = spec.rows_slice(r, r + 1)
        ref = oracle.vlb_compress(row)
        assert y[r] == oracle.vlb_matvec(ref, x)[0], r
        # the row's bits under the whole matrix's k
        assert rb[r + 1] - rb[r] == ref.nbits - spec.cols * ref.k + spec.cols * g.k, r
        for j in (0, 31, 32, spec.cols - 1):
            assert c.vlb_get(g, r, j) == int(row[0, j])


@pytest.mark.parametrize("shape", [(7, 1000), (2, 16384), (3, 16416), (40, 2000)], ids=str)
def test_rare_wide_pairs(shape):
    """Mostly short pairs with a few past 32 bits: the staged kernel's
    short-pair walk with its long-pair branch (the four-word walk is for
    matrices whose pairs average more than 24 bits)."""
    c = ccm()
    rng = np.random.default_rng(shape[1])
    A = rng.integers(0, 8, size=shape, dtype=np.int64)
    flat = A.reshape(-1)
    wide = rng.choice(flat.size, size=max(3, flat.size // 100), replace=False)
    flat[wide] = rng.integers(1 << 30, 1 << 62, size=wide.size, dtype=np.int64)
    for signed in (False, True):
        M = A if not signed else np.where(rng.random(A.shape) < 0.5, -A - 1, A)
        ref = oracle.vlb_compress(M)
        assert ref.nbits < 24 * M.size
        g = c.vlb_compress(dev(M))
        check_encoding(g, ref)
        check_ops(g, ref, M, rng)
