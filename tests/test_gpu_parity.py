"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer results are compared bit-exactly: compressed results by their header
and canonical payload bytes, vectors element by element.  Small cases span
several tiles and ragged tails; the workload-sized cases are checked on
sampled rows and entries the oracle computes one by one.
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


def assert_same_packed(gpu, ref):
    assert gpu.header() == oracle.header(ref)
    assert gpu.payload_bytes() == ref.payload_bytes()
    # every byte of the capacity past the canonical payload is written as zero
    tail = gpu.payload[8 * gpu.words:].cpu().numpy()
    assert not tail.any()


SHAPES = [(1, 1), (1, 33), (3, 37), (65, 33), (130, 257), (7, 1000)]


@pytest.mark.parametrize("b", list(range(1, 65)))
def test_compress_decompress_all_widths(b):
    c = ccm()
    rng = np.random.default_rng(100 + b)
    for signed in ((False, True) if b < 64 else (True,)):
        for rows, cols in SHAPES[: 3 + b % 4]:
            if signed and b == 1 and rows * cols < 2:
                continue
            m = rand_matrix(rng, rows, cols, b, signed)
            ref = oracle.compress(m)
            g = c.compress(dev(m))
            assert_same_packed(g, ref)
            assert np.array_equal(c.decompress(g).cpu().numpy(), oracle.decompress(ref))
            if b <= 31:
                g32 = c.compress(dev(m, torch.int32))
                assert_same_packed(g32, ref)


def test_worked_example_on_gpu():
    c = ccm()
    vals = np.array([[900, 1023, 721, 256, 1, 10, 700, 20]])
    g = c.compress(dev(vals))
    ref = oracle.compress(vals)
    assert_same_packed(g, ref)
    assert [c.get(g, 0, j) for j in range(8)] == vals[0].tolist()


def test_get_and_gather():
    c = ccm()
    rng = np.random.default_rng(7)
    for b, signed in ((3, False), (10, False), (33, True), (64, True), (17, True)):
        m = rand_matrix(rng, 45, 71, b, signed)
        ref = oracle.compress(m)
        g = c.compress(dev(m))
        for _ in range(20):
            i, j = int(rng.integers(0, 45)), int(rng.integers(0, 71))
            assert c.get(g, i, j) == oracle.get(ref, i, j)
        ii = rng.integers(0, 45, size=1000)
        jj = rng.integers(0, 71, size=1000)
        vals, bad = c.gather(g, dev(ii), dev(jj))
        assert not bad
        assert vals.cpu().numpy().tolist() == [oracle.get(ref, int(i), int(j))
                                               for i, j in zip(ii, jj)]
        vals, bad = c.gather(g, dev(np.array([0, 45, 3])), dev(np.array([0, 0, -1])))
        assert bad and vals.cpu().numpy().tolist()[1:] == [0, 0]
        with pytest.raises(c.CcmError):
            c.get(g, 45, 0)
        with pytest.raises(c.CcmError):
            c.get(g, 0, -1)


ADD_CASES = [(1, False, 1, False), (3, True, 5, False), (10, False, 10, False),
             (12, True, 12, True), (31, True, 30, False), (33, False, 2, True),
             (40, True, 63, False), (64, True, 7, True), (62, False, 62, False)]


@pytest.mark.parametrize("onepass", [True, False], ids=["onepass", "plan"])
@pytest.mark.parametrize("ba,sa,bb,sb", ADD_CASES)
def test_add_matches_oracle(ba, sa, bb, sb, onepass):
    c = ccm()
    rng = np.random.default_rng(ba * 100 + bb)
    for rows, cols in ((1, 1), (5, 77), (70, 130)):
        A = rand_matrix(rng, rows, cols, ba, sa)
        B = rand_matrix(rng, rows, cols, bb, sb)
        try:
            ref = oracle.add(oracle.compress(A), oracle.compress(B))
        except oracle.OracleError as e:
            assert e.code == oracle.E_OVERFLOW
            with pytest.raises(c.CcmError) as ei:
                c.add(c.compress(dev(A)), c.compress(dev(B)), onepass=onepass)
            assert ei.value.status == c._lib.E_OVERFLOW
            continue
        assert_same_packed(c.add(c.compress(dev(A)), c.compress(dev(B)), onepass=onepass), ref)


# Operands of one width and signedness whose sums need one more bit: the
# one-pass add's compile-time kernel, at every width it covers (b <= 15),
# over many packing blocks and a ragged last group, with each operand's
# extremes present (so the sums reach both ends of their bound).
@pytest.mark.parametrize("b", list(range(1, 16)))
def test_add_same_width_every_b(b):
    c = ccm()
    rng = np.random.default_rng(4000 + b)
    for signed in (False, True):
        for rows, cols in ((300, 1001), (3, 37)):
            A = rand_matrix(rng, rows, cols, b, signed)
            B = rand_matrix(rng, rows, cols, b, signed)
            lo, hi = ((-(1 << (b - 1)), (1 << (b - 1)) - 1) if signed else (0, (1 << b) - 1))
            A.reshape(-1)[-1], B.reshape(-1)[-1] = hi, hi
            A.reshape(-1)[0], B.reshape(-1)[0] = lo, lo
            ref = oracle.add(oracle.compress(A), oracle.compress(B))
            for onepass in (True, False):
                g = c.add(c.compress(dev(A)), c.compress(dev(B)), onepass=onepass)
                assert g.bits == b + 1, (b, signed, rows, cols)
                assert_same_packed(g, ref)
            pend = c.add_async(c.compress(dev(A)), c.compress(dev(B)))
            assert_same_packed(pend.get(), ref)


# Operand ranges at the edges of the 32-bit elementwise classes (every operand
# and result in int32, or all non-negative with results below 2^32) and just
# past them, so each class and the int64 path meet their boundary values.
EDGE_PAIRS = [
    ((-2**31, 0), (0, 2**31 - 1)),            # int32 class, result spans int32
    ((-2**31, -1), (-1, 0)),                  # result reaches -2^31 - 1: int64
    ((0, 2**32 - 1), (0, 0)),                 # uint32 class, result up to 2^32 - 1
    ((0, 2**31), (0, 2**31 - 1)),             # uint32 class, result 2^32 - 1
    ((0, 2**32 - 1), (0, 1)),                 # result 2^32: int64
    ((-5, 2**31 - 1), (0, 1)),                # result 2^31 with a signed operand: int64
]


@pytest.mark.parametrize("onepass", [True, False], ids=["onepass", "plan"])
@pytest.mark.parametrize("ra,rb", EDGE_PAIRS)
def test_add_class_edges(ra, rb, onepass):
    c = ccm()
    rng = np.random.default_rng(abs(ra[0]) % 97 + rb[1] % 89)
    for rows, cols in ((3, 40), (65, 97)):
        A = rng.integers(ra[0], ra[1], size=(rows, cols), endpoint=True, dtype=np.int64)
        B = rng.integers(rb[0], rb[1], size=(rows, cols), endpoint=True, dtype=np.int64)
        # both extremes of each operand, paired so the result extremes occur too
        A.flat[0], B.flat[0] = ra[0], rb[0]
        A.flat[1], B.flat[1] = ra[1], rb[1]
        ref = oracle.add(oracle.compress(A), oracle.compress(B))
        assert_same_packed(c.add(c.compress(dev(A)), c.compress(dev(B)), onepass=onepass), ref)


@pytest.mark.parametrize("r,s", [((-2**31, 2**31 - 1), 1), ((-2**31, 2**31 - 1), -1),
                                 ((-2**15, 2**15 - 1), 2**16), ((0, 2**16 - 1), 2**16 + 1),
                                 ((0, 2**31 - 1), 2), ((0, 2**32 - 1), 1), ((-7, 9), -(2**28))])
def test_scale_class_edges(r, s):
    c = ccm()
    rng = np.random.default_rng(r[1] % 1000 + abs(s) % 1000)
    A = rng.integers(r[0], r[1], size=(17, 70), endpoint=True, dtype=np.int64)
    A.flat[0], A.flat[1] = r[0], r[1]
    ref = oracle.scale(oracle.compress(A), s)
    assert_same_packed(c.scale(c.compress(dev(A)), s), ref)


@pytest.mark.parametrize("shape", [(1, 5), (5, 77), (70, 130), (3, 96)], ids=str)
def test_elementwise_extremes_in_last_group(shape):
    """The result's minimum and maximum only in the last (ragged, when n % 32
    != 0) group: the range pass must see them there."""
    c = ccm()
    rng = np.random.default_rng(shape[1])
    A = rng.integers(0, 100, size=shape, dtype=np.int64)
    B = rng.integers(0, 100, size=shape, dtype=np.int64)
    A.flat[-1] = 1 << 20
    B.flat[-2 if A.size > 1 else -1] = -5
    ref = oracle.add(oracle.compress(A), oracle.compress(B))
    for onepass in (True, False):
        assert_same_packed(c.add(c.compress(dev(A)), c.compress(dev(B)), onepass=onepass), ref)
    for s in (3, -3):
        assert_same_packed(c.scale(c.compress(dev(A)), s), oracle.scale(oracle.compress(A), s))


@pytest.mark.parametrize("onepass", [True, False], ids=["onepass", "plan"])
def test_add_overflow_and_shape(onepass):
    c = ccm()
    a = c.compress(dev(np.array([[2**63 - 1, 0]])))
    one = c.compress(dev(np.array([[1, 0]])))
    with pytest.raises(c.CcmError) as ei:
        c.add(a, one, onepass=onepass)
    assert ei.value.status == c._lib.E_OVERFLOW
    with pytest.raises(c.CcmError) as ei:
        c.add(a, c.compress(dev(np.array([[1], [0]]))), onepass=onepass)
    assert ei.value.status == c._lib.E_SHAPE


# One-pass add: the width the headers bound against the exact one.
ONEPASS_CASES = {
    # extremes of A and B at different positions: bound [0, 2000] (11 bits),
    # exact [0, 1000] (10 bits), so the sums are packed a second time
    "loose_bound_repack": lambda r, n: (np.where(np.arange(n) == 0, 1000, r.integers(0, 500, n)),
                                        np.where(np.arange(n) == n - 1, 1000,
                                                 r.integers(0, 500, n))),
    # bound [-5, 110] (signed, 8 bits), exact [0, 100] (unsigned, 7 bits)
    "sign_changes": lambda r, n: (np.where(np.arange(n) == 0, -5, r.integers(0, 91, n)),
                                  np.where(np.arange(n) == 0, 5, r.integers(0, 11, n))),
    # bound equals the exact range: one pass
    "tight_bound": lambda r, n: (r.integers(-2**14, 2**14, n), r.integers(-2**14, 2**14, n)),
    # unsigned 32-bit class at its top: sums up to 2^32 - 1
    "u32_top": lambda r, n: (r.integers(0, 2**31 + 1, n), r.integers(0, 2**31, n)),
    # int64 class, extremes apart: bound [0, 2^41] (42 bits), exact 41 bits
    "i64_loose_bound": lambda r, n: (np.where(np.arange(n) == 0, 2**40, r.integers(0, 2**39, n)),
                                     np.where(np.arange(n) == n - 1, 2**40,
                                              r.integers(0, 2**39, n))),
    # int64 class, signed, the bound's width reached
    "i64_tight_bound": lambda r, n: (r.integers(-2**45, 2**45, n), r.integers(-2**45, 2**45, n)),
    # a 64-bit result: bound [-2^62 - 2^61, 2^62 + 2^61 - 2] inside int64
    "i64_full_width": lambda r, n: (r.integers(-2**62, 2**62, n), r.integers(-2**61, 2**61, n)),
    # a bound past int64 whose sums fit: the range pass runs first
    "bound_past_int64": lambda r, n: (np.where(np.arange(n) % 2 == 0, 2**62 + 7, -(2**62)),
                                      np.where(np.arange(n) % 2 == 0, -(2**62), 2**62 + 5)),
}


@pytest.mark.parametrize("case", sorted(ONEPASS_CASES))
@pytest.mark.parametrize("shape", [(1, 1), (3, 37), (300, 1001)], ids=str)
def test_add_onepass_bound_cases(case, shape):
    """Several blocks (300 x 1001 is 9385 groups, the last ragged) fold the
    exact range; each case's result must equal the oracle's bit for bit."""
    c = ccm()
    n = shape[0] * shape[1]
    rng = np.random.default_rng(len(case) * 7 + n)
    a, b = ONEPASS_CASES[case](rng, n)
    A = np.asarray(a, dtype=np.int64).reshape(shape)
    B = np.asarray(b, dtype=np.int64).reshape(shape)
    ref = oracle.add(oracle.compress(A), oracle.compress(B))
    got = c.add(c.compress(dev(A)), c.compress(dev(B)), onepass=True)
    assert_same_packed(got, ref)
    assert_same_packed(c.add(c.compress(dev(A)), c.compress(dev(B)), onepass=False), ref)


# The one-pass add folds each packing block's extremes (8192 elements per
# block) into one of 64 range slots (block i into slot i mod 64), and a block
# issues its atomic only when its extreme beats the value it reads in its
# slot.  2048 x 4096 is 1024 blocks, 16 per slot: these patterns put the
# extremes where that skip decides the result.
_NB = 8192


def _blk(n):
    return np.arange(n, dtype=np.int64) // _NB


def _peak(n):
    e = np.arange(n, dtype=np.int64)
    return (e % _NB == 5) & ((_blk(n) % 7 == 0) | (_blk(n) == n // _NB - 1))


LATE_EXTREME_CASES = {
    # every block's maximum beats all earlier blocks' (no skip for the max),
    # every block's minimum is above block 0's (skips for the min)
    "increasing": lambda r, n: (_blk(n) * 3 + r.integers(0, 3, n), r.integers(0, 3, n)),
    # the reverse: the exact minimum only in the last block
    "decreasing": lambda r, n: ((1023 - _blk(n)) * 3 + r.integers(0, 3, n), r.integers(0, 3, n)),
    # random values with a spike in block 1000 (slot 40, written by 15 earlier
    # blocks) and a dip in block 900 (slot 4)
    "late_spikes": lambda r, n: (np.where(np.arange(n) == 1000 * _NB + 17, 5000,
                                          r.integers(0, 1000, n)),
                                 np.where(np.arange(n) == 900 * _NB + 3, -3000,
                                          r.integers(0, 1000, n))),
    # the same maximum reached in every seventh block and in the last one
    "repeated_extremes": lambda r, n: (np.where(_peak(n), 700, 350),
                                       np.where(_peak(n), 300, r.integers(0, 300, n))),
}


@pytest.mark.parametrize("scale", [1, 2**35], ids=["i32_class", "i64_class"])
@pytest.mark.parametrize("case", sorted(LATE_EXTREME_CASES))
def test_add_onepass_skip_fold(case, scale):
    """Thousands of packing blocks per add: the exact extremes folded with
    skipped atomics must still be the true ones (header and payload equal the
    oracle's byte for byte), for both value classes."""
    c = ccm()
    shape = (2048, 4096)
    n = shape[0] * shape[1]
    rng = np.random.default_rng(len(case) * 11 + (scale > 1))
    a, b = LATE_EXTREME_CASES[case](rng, n)
    A = (np.asarray(a, dtype=np.int64) * scale).reshape(shape)
    B = (np.asarray(b, dtype=np.int64) * scale).reshape(shape)
    ref = oracle.add(oracle.compress(A), oracle.compress(B))
    got = c.add(c.compress(dev(A)), c.compress(dev(B)), onepass=True)
    assert (got.vmin, got.vmax) == (int((A + B).min()), int((A + B).max()))
    assert_same_packed(got, ref)


@pytest.mark.parametrize("b,signed", [(1, False), (4, True), (13, False), (31, True),
                                      (40, False), (64, True)])
def test_scale_matches_oracle(b, signed):
    c = ccm()
    rng = np.random.default_rng(b)
    A = rand_matrix(rng, 33, 65, b, signed)
    pa = oracle.compress(A)
    ga = c.compress(dev(A))
    for s in (0, 1, -1, 7, -3, 2**20, -(2**30)):
        try:
            ref = oracle.scale(pa, s)
        except oracle.OracleError as e:
            assert e.code == oracle.E_OVERFLOW
            with pytest.raises(c.CcmError):
                c.scale(ga, s)
            continue
        assert_same_packed(c.scale(ga, s), ref)


MV_SHAPES = [(1, 1), (1, 40), (17, 31), (33, 96), (100, 257), (3, 9000), (70, 16500)]
# cols % 128 == 0: rows start on 16-byte boundaries (the aligned b <= 15 path);
# 8320 leaves one lane a second quad of groups, 16384 is one full panel with
# two quads per lane, 16512 = 16384 + 128 spans two column panels
MV_ALIGNED = [(5, 128), (37, 256), (130, 1024), (9, 8320), (3, 16384), (11, 16512)]


@pytest.mark.parametrize("b", list(range(1, 65)))
def test_matvec_all_widths(b):
    c = ccm()
    rng = np.random.default_rng(1000 + b)
    for signed in ((False, True) if b < 64 else (True,)):
        shapes = MV_SHAPES if b in (1, 3, 7, 10, 12, 17, 31, 32, 33, 64) else MV_SHAPES[:5]
        shapes = shapes + (MV_ALIGNED if b <= 16 else MV_ALIGNED[:1])
        for rows, cols in shapes:
            if signed and b == 1 and rows * cols < 2:
                continue
            A = rand_matrix(rng, rows, cols, b, signed)
            pa = oracle.compress(A)
            g = c.compress(dev(A))
            x16 = rng.integers(-(1 << 15), 1 << 15, size=cols)
            x32 = rng.integers(-(1 << 31), 1 << 31, size=cols)
            x64 = rng.integers(-(1 << 63), (1 << 63) - 1, size=cols, endpoint=True)
            for x, dt in ((x16, torch.int32), (x32, torch.int32), (x64, torch.int64)):
                y = c.matvec(g, dev(x, dt)).cpu().numpy()
                assert np.array_equal(y, oracle.matvec(pa, x)), (b, signed, rows, cols, dt)


# Fields at their largest magnitudes against x at the ends of the int16 range,
# on the aligned kernel's shapes: the exact 32-bit sums of the int16-x paths
# (digit products at b <= 4, 24-bit multiply-add runs above) at their bounds.
@pytest.mark.parametrize("b", list(range(1, 16)))
def test_matvec_int16_x_extremes(b):
    c = ccm()
    shapes = [(37, 16512)] + ([(9, 8320), (130, 1024)] if b <= 4 else [])
    for signed in (False, True):
        lo, hi = ((-(1 << (b - 1)), (1 << (b - 1)) - 1) if signed else (0, (1 << b) - 1))
        if b == 1 and signed:
            lo, hi = -1, 0
        for rows, cols in shapes:
            j = np.arange(cols)
            fields = {"max": np.full((rows, cols), hi), "min": np.full((rows, cols), lo),
                      "alternate": np.broadcast_to(np.where(j % 2 == 0, hi, lo), (rows, cols))}
            xs = {"-2^15": np.full(cols, -(1 << 15)), "2^15-1": np.full(cols, (1 << 15) - 1),
                  "alternate": np.where(j % 2 == 0, (1 << 15) - 1, -(1 << 15))}
            for fname, A in fields.items():
                if not signed and fname == "min":
                    continue
                A = np.ascontiguousarray(A, dtype=np.int64)
                pa = oracle.compress(A)
                g = c.compress(dev(A))
                assert g.header() == oracle.header(pa), (b, signed, fname)
                for xname, x in xs.items():
                    y = c.matvec(g, dev(x, torch.int32)).cpu().numpy()
                    assert np.array_equal(y, oracle.matvec(pa, x)), (b, signed, rows, cols,
                                                                     fname, xname)


# Column counts that are not a multiple of 128 (rows start at any bit): the
# aligned kernel's ragged form at b <= 4, whose units fetch 16-byte-aligned
# supersets of each quad and shift them into place, the general kernel at
# 5..8 and the wide kernel at 16 and up.  One, two and three column panels
# (the grid shared by panels of unequal width) up to seven (100001 columns;
# 98304 = six whole panels), panels that end inside a group, x zero-padded to
# whole quads.
MV_RAGGED = [(1, 1), (3, 127), (37, 129), (5, 16383), (9, 16385), (4, 32845), (130, 1000),
             (1000, 130), (2, 77), (3, 100001), (2, 98304)]


@pytest.mark.parametrize("b", list(range(1, 9)) + [16, 17, 24, 31])
def test_matvec_ragged_columns(b):
    c = ccm()
    rng = np.random.default_rng(3000 + b)
    for signed in (False, True):
        for rows, cols in MV_RAGGED:
            if signed and b == 1 and rows * cols < 2:
                continue
            A = rand_matrix(rng, rows, cols, b, signed)
            pa = oracle.compress(A)
            g = c.compress(dev(A))
            x16 = rng.integers(-(1 << 15), (1 << 15) - 1, size=cols, endpoint=True)
            x16[int(rng.integers(0, cols))] = -(1 << 15)
            x16[int(rng.integers(0, cols))] = (1 << 15) - 1
            x17 = x16.copy()
            x17[int(rng.integers(0, cols))] = 1 << 15  # one value outside int16
            x32 = rng.integers(-(1 << 31), 1 << 31, size=cols)
            for x in (x16, x17, x32):
                y = c.matvec(g, dev(x, torch.int32)).cpu().numpy()
                assert np.array_equal(y, oracle.matvec(pa, x)), (b, signed, rows, cols)
        # fields at their largest magnitudes against x at both ends of int16
        lo, hi = ((-(1 << (b - 1)), (1 << (b - 1)) - 1) if signed else (0, (1 << b) - 1))
        if b == 1 and signed:
            lo, hi = -1, 0
        for rows, cols in ((7, 16385), (3, 32845)):
            j = np.arange(cols)
            A = np.ascontiguousarray(np.broadcast_to(np.where(j % 3 == 0, lo, hi), (rows, cols)),
                                     dtype=np.int64)
            pa = oracle.compress(A)
            g = c.compress(dev(A))
            for x in (np.full(cols, -(1 << 15)), np.full(cols, (1 << 15) - 1),
                      np.where(j % 2 == 0, (1 << 15) - 1, -(1 << 15))):
                y = c.matvec(g, dev(x, torch.int32)).cpu().numpy()
                assert np.array_equal(y, oracle.matvec(pa, x)), (b, signed, rows, cols, "extremes")


# operands whose values fit int8 take the MFMA path (unsigned b <= 7, signed b <= 8)
@pytest.mark.parametrize("ba,sa,bb,sb", [(10, False, 10, False), (6, False, 4, True),
                                         (1, False, 1, True), (20, True, 17, False),
                                         (33, True, 20, False), (8, False, 8, True),
                                         (7, False, 8, True), (8, True, 3, False),
                                         (2, True, 5, True)])
def test_matmul_matches_oracle(ba, sa, bb, sb):
    c = ccm()
    rng = np.random.default_rng(ba * 7 + bb)
    # ragged in every dimension, up to several 256 x 256 tiles and K chunks of 64
    for M, K, N in ((1, 1, 1), (5, 7, 3), (65, 33, 70), (130, 100, 129), (257, 300, 131),
                    (128, 64, 128), (300, 200, 520), (513, 130, 257)):
        A = rand_matrix(rng, M, K, ba, sa)
        B = rand_matrix(rng, K, N, bb, sb)
        pa, pb = oracle.compress(A), oracle.compress(B)
        ref = oracle.matmul(pa, pb)
        assert_same_packed(c.matmul(c.compress(dev(A)), c.compress(dev(B))), ref)


# every operand width and sign the int8 MFMA path decodes (values fit int8:
# unsigned b <= 7, signed b <= 8), on both sides of the product
I8_WIDTHS = [(b, False) for b in range(1, 8)] + [(b, True) for b in range(1, 9)]


@pytest.mark.parametrize("b,signed", I8_WIDTHS)
def test_matmul_i8_every_width(b, signed):
    c = ccm()
    rng = np.random.default_rng(500 + 2 * b + signed)
    ob, osg = I8_WIDTHS[(I8_WIDTHS.index((b, signed)) + 5) % len(I8_WIDTHS)]
    for M, K, N in ((70, 150, 90), (33, 64, 260)):
        for A, B in ((rand_matrix(rng, M, K, b, signed), rand_matrix(rng, K, N, ob, osg)),
                     (rand_matrix(rng, M, K, ob, osg), rand_matrix(rng, K, N, b, signed))):
            pa, pb = oracle.compress(A), oracle.compress(B)
            assert_same_packed(c.matmul(c.compress(dev(A)), c.compress(dev(B))),
                               oracle.matmul(pa, pb))


@pytest.mark.parametrize("ba,sa,bb,sb", [(6, False, 4, True), (1, True, 8, True), (7, False, 2, False)])
def test_matmul_i8_many_tiles(ba, sa, bb, sb):
    """4 x 2 output tiles (a count the XCD-grouped tile order remaps), every
    dimension ragged, three K steps, against the oracle byte for byte."""
    c = ccm()
    rng = np.random.default_rng(900 + ba + 10 * bb)
    A = rand_matrix(rng, 1000, 300, ba, sa)
    B = rand_matrix(rng, 300, 500, bb, sb)
    assert_same_packed(c.matmul(c.compress(dev(A)), c.compress(dev(B))),
                       oracle.matmul(oracle.compress(A), oracle.compress(B)))


def test_matmul_overflow_rule():
    c = ccm()
    a = c.compress(dev(np.array([[2**31, 2**31]])))
    b = c.compress(dev(np.array([[2**31], [-2**31]])))
    with pytest.raises(c.CcmError) as ei:
        c.matmul(a, b)
    assert ei.value.status == c._lib.E_OVERFLOW
    with pytest.raises(c.CcmError) as ei:
        c.matmul(a, a)
    assert ei.value.status == c._lib.E_SHAPE


def test_serialize_round_trip():
    c = ccm()
    rng = np.random.default_rng(5)
    A = rand_matrix(rng, 19, 23, 21, True)
    g = c.compress(dev(A))
    blob = g.serialize()
    assert blob == oracle.header(oracle.compress(A)) + oracle.compress(A).payload_bytes()
    back = c.from_serialized(blob)
    assert np.array_equal(c.decompress(back).cpu().numpy(), A)


def test_device_generator_matches_host_twin():
    c = ccm()
    for dt, lo, hi in ((torch.int64, -(1 << 31), 1 << 31), (torch.int32, -(1 << 15), 1 << 15),
                       (torch.int64, 0, 1 << 32), (torch.int64, 5, 6), (torch.int32, 0, 1000)):
        t = torch.empty(100003, dtype=dt, device="cuda")
        c.fill_uniform(t, lo, hi, seed=W.seed_for(9, 1), stream_id=3, start=17)
        want = W.uniform(W.seed_for(9, 1), 3, 17, 100003, lo, hi)
        assert np.array_equal(t.cpu().numpy().astype(np.int64), want)
    m = c.generate(301, 77, -100, 1 << 20, seed=W.seed_for(9, 2), stream_id=5)
    ref = oracle.compress(W.uniform_matrix(W.seed_for(9, 2), 5, 301, 77, -100, 1 << 20))
    assert_same_packed(m, ref)


def test_small_plain_workload_full():
    """256x256 in [0, 2^10): every operation checked in full."""
    c = ccm()
    a_s, b_s, x_s, s = W.small_plain()
    A, B, x = a_s.dense(), b_s.dense(), x_s.dense()
    pa, pb = oracle.compress(A), oracle.compress(B)
    ga, gb = c.compress(dev(A)), c.compress(dev(B))
    assert ga.bits == 10
    assert_same_packed(ga, pa)
    assert_same_packed(gb, pb)
    assert np.array_equal(c.decompress(ga).cpu().numpy(), A)
    rng = np.random.default_rng(W.seed_for(1, 3))
    ii, jj = rng.integers(0, 256, 1000), rng.integers(0, 256, 1000)
    vals, bad = c.gather(ga, dev(ii), dev(jj))
    assert not bad and vals.cpu().numpy().tolist() == [oracle.get(pa, int(i), int(j))
                                                       for i, j in zip(ii, jj)]
    assert np.array_equal(c.matvec(ga, dev(x)).cpu().numpy(), oracle.matvec(pa, x))
    assert_same_packed(c.add(ga, gb), oracle.add(pa, pb))
    assert_same_packed(c.scale(ga, s), oracle.scale(pa, s))
    gm = c.matmul(ga, gb)
    assert_same_packed(gm, oracle.matmul(pa, pb))
    # the same values as plain int64 arithmetic
    assert np.array_equal(c.decompress(gm).cpu().numpy(), A @ B)
