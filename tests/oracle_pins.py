"""Pins of the CPU oracle to facts other than the oracle itself.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError if
the oracle disagrees with what the paper or the mathematics fixes:

* values the paper prints (Table 1, Eq. 1, the worked examples of Method 1
  and Method 2 and the bitstring count), read from ``tests/golden/``;
* closed forms (the word count, Eq. 15's bits-used relation);
* invariants (round trips, minimality of the width, zero padding, locality of
  the encoding);
* brute force against uncompressed Python integer arithmetic on tiny inputs,
  exhaustive for 2x2 matrices of 2-bit values;
* algebraic identities of the operations.

``tests/test_oracle_pins.py`` runs them on the oracle; the mutation test runs
them on deliberately broken builds of the oracle source and requires each
build to fail at least one of them.
"""
from __future__ import annotations

import itertools
import math
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
M64 = (1 << 64) - 1


def _golden_kv(name: str) -> dict:
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=", 1)
            out[k.strip()] = v.strip()
    return out


def _table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_bitlengths.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                v, binary, bl = line.split()
                rows.append((int(v), binary, int(bl)))
    return rows


def _to_signed64(u: int) -> int:
    u &= M64
    return u - (1 << 64) if u >> 63 else u


def _min_width(lo: int, hi: int) -> tuple[int, bool]:
    """Smallest width holding [lo, hi], searched by brute force over b."""
    signed = lo < 0
    for b in range(1, 65):
        if signed:
            if -(1 << (b - 1)) <= lo and hi < (1 << (b - 1)):
                return b, True
        else:
            if hi < (1 << b):
                return b, False
    raise AssertionError("no width")


# ---------------------------------------------------------------------------
# bit-length and width
# ---------------------------------------------------------------------------

def pin_table1(o):
    """Table 1: bit-lengths of the eight printed elements (Eq. 1)."""
    for v, binary, bl in _table1():
        assert int(binary, 2) == v and len(binary) == bl
        assert o.sm_width(v) == bl, (v, o.sm_width(v), bl)
        assert o.width(0, v) == (bl, False)


def pin_eq1_special_case(o):
    """Eq. 1: sup M in {0, 1} needs one bit; all-zero and all-one matrices get b = 1."""
    assert o.sm_width(0) == 1 and o.sm_width(1) == 1
    assert o.width(0, 0) == (1, False) and o.width(1, 1) == (1, False)
    for fill in (0, 1):
        p = o.compress(np.full((3, 5), fill, dtype=np.int64))
        assert p.bits == 1 and not p.is_signed
        assert o.decompress(p).tolist() == np.full((3, 5), fill).tolist()


def pin_bitlen_bruteforce(o):
    """bitlen against Python's int.bit_length on all u < 2^14 and at every 2^t +- 1."""
    for u in range(1 << 14):
        assert o.bitlen(u) == u.bit_length(), u
    for t in range(64):
        for u in ((1 << t) - 1, 1 << t, (1 << t) + 1):
            if u <= M64:
                assert o.bitlen(u) == u.bit_length(), u
    assert o.bitlen(M64) == 64


def pin_width_bruteforce(o):
    """The width rule equals a brute-force search for the smallest holding width."""
    rng = np.random.default_rng(7)
    cases = [(0, 0), (0, 1), (-1, 0), (-1, -1), (-2, 1), (-3, 0), (0, 2**63 - 1),
             (-2**63, 2**63 - 1), (-2**63, -2**63), (-2**63, 0), (5, 5), (-129, 127),
             (-128, 127), (-128, 128)]
    for t in range(1, 63):
        cases += [(0, (1 << t) - 1), (0, 1 << t), (-(1 << t), (1 << t) - 1),
                  (-(1 << t) - 1, 0), (-(1 << t), 1 << t)]
    for _ in range(300):
        a, b = sorted(int(v) for v in rng.integers(-2**63, 2**63 - 1, size=2, endpoint=True))
        sh = int(rng.integers(0, 63))
        cases.append((a >> sh, b >> sh))
    for lo, hi in cases:
        assert o.width(lo, hi) == _min_width(lo, hi), (lo, hi)


# ---------------------------------------------------------------------------
# encoding
# ---------------------------------------------------------------------------

def pin_worked_example(o):
    """Method 1's worked example: the two bitstrings of Eq. 3 and the straddle step."""
    g = _golden_kv("sm_worked_example.txt")
    vals = [int(v) for v in g["values"].split()]
    w0 = int(g["bitstring_1"].replace(" ", ""), 2)
    w1 = int(g["bitstring_2"].replace(" ", ""), 2)
    p = o.compress(np.array([vals], dtype=np.int64))
    assert p.bits == int(g["bits"]) and not p.is_signed
    assert p.words == int(g["words"]) == o.words(1, 8, 10)
    assert [int(w) for w in p.payload] == [w0, w1]
    # the same bytes read as 32-bit words, little-endian
    w32 = np.frombuffer(p.payload_bytes(), dtype="<u4").tolist()
    assert w32 == [w0 & 0xFFFFFFFF, w0 >> 32, w1 & 0xFFFFFFFF, w1 >> 32]
    assert o.decompress(p).tolist() == [vals]
    assert [o.get(p, 0, j) for j in range(8)] == vals
    h = o.header(p)
    assert h[:4] == b"CCM1" and h[4:6] == b"\x01\x00" and h[6] == 10 and h[7] == 0
    le = lambda a, b: int.from_bytes(h[a:b], "little", signed=True)
    assert (le(8, 16), le(16, 24), le(24, 32), le(32, 40), le(40, 48)) == (1, 8, 1, 1023, 2)
    assert h[48:] == bytes(16)


def pin_signed_headers(o):
    """The header and bitstring of a small signed matrix, row-major and
    column-major, against bytes derived by hand: flags 1 and 3, the negative
    min in little-endian two's complement, 4-bit two's complement fields."""
    g = _golden_kv("signed_headers.txt")
    A = np.array([[int(v) for v in r.split()] for r in g["matrix"].split(";")], dtype=np.int64)
    hx = lambda key: bytes(int(t, 16) for t in g[key].split())
    p = o.compress(A)
    assert (p.bits, p.is_signed) == (int(g["bits"]), True)
    assert o.header(p) == hx("header_row_major")
    assert [int(w) for w in p.payload] == [int(g["payload_row_major"], 16)]
    q = o.compress_cm(A)
    assert (q.bits, q.is_signed) == (int(g["bits"]), True)
    assert o.header_cm(q) == hx("header_col_major")
    assert [int(w) for w in q.payload] == [int(g["payload_col_major"], 16)]
    assert o.decompress(p).tolist() == A.tolist() == o.decompress_cm(q).tolist()


def pin_word_count(o):
    """floor(n*b/64) + 1 bitstrings; the payload uses exactly n*b bits (Eq. 15)."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        r, c, b = int(rng.integers(1, 1000)), int(rng.integers(1, 1000)), int(rng.integers(1, 65))
        assert o.words(r, c, b) == (r * c * b) // 64 + 1
        assert o.packed_bytes(r, c, b) == 64 + 8 * ((r * c * b) // 64 + 1)
    # n*b a multiple of 64: the paper's formula still adds one (zero) bitstring
    assert o.words(8, 8, 1) == 2 and o.words(1, 64, 1) == 2
    for b in range(1, 65):
        # Eq. 15: eta_1 = (64 - b) / 64 from the bits used, n*b
        n = 64
        assert (64 * n - n * b) / (64 * n) == (64 - b) / 64


def _random_matrix(rng, rows, cols, b, signed):
    if signed:
        lo, hi = -(1 << (b - 1)), (1 << (b - 1)) - 1
    else:
        lo, hi = 0, (1 << b) - 1
    vals = rng.integers(lo, hi, size=(rows, cols), endpoint=True, dtype=np.int64)
    # force the extremes in so the width is exactly b
    flat = vals.reshape(-1)
    flat[int(rng.integers(0, flat.size))] = hi
    if signed:
        flat[int(rng.integers(0, flat.size))] = lo
    return vals


def _field_bits(p, e):
    """Field e of p read from the payload bytes with Python big integers."""
    big = int.from_bytes(p.payload_bytes(), "little")
    return (big >> (e * p.bits)) & ((1 << p.bits) - 1)


def pin_round_trip(o):
    """compress -> decompress is the identity; size, padding and minimality hold."""
    rng = np.random.default_rng(5)
    shapes = [(1, 1), (1, 7), (7, 1), (3, 21), (64, 1), (2, 32), (5, 13), (17, 19), (1, 200)]
    for b in range(1, 65):
        for signed in ((False, True) if b < 64 else (True,)):
            for rows, cols in shapes[int(rng.integers(0, 3)):][:4]:
                if b == 1 and signed and rows * cols < 2:
                    continue
                m = _random_matrix(rng, rows, cols, b, signed)
                p = o.compress(m)
                lo, hi = int(m.min()), int(m.max())
                assert (p.vmin, p.vmax) == (lo, hi)
                assert (p.bits, p.is_signed) == _min_width(lo, hi), (b, signed)
                assert p.words == (rows * cols * p.bits) // 64 + 1
                assert np.array_equal(o.decompress(p), m)
                # every field holds the low b bits of the value's two's complement
                for e in (0, rows * cols // 2, rows * cols - 1):
                    v = int(m.reshape(-1)[e])
                    assert _field_bits(p, e) == v & ((1 << p.bits) - 1)
                # bits past n*b are zero
                big = int.from_bytes(p.payload_bytes(), "little")
                assert big >> (rows * cols * p.bits) == 0


def pin_signed_small_bruteforce(o):
    """Every value of every width up to 5 bits, alone and in pairs, round-trips."""
    for b in range(1, 6):
        vals = list(range(-(1 << (b - 1)), 1 << (b - 1))) if b > 0 else []
        for v in vals:
            p = o.compress(np.array([[v]], dtype=np.int64))
            assert o.decompress(p)[0, 0] == v
            assert p.bits == _min_width(v, v)[0]
        for v, w in itertools.product(vals, repeat=2):
            m = np.array([[v, w]], dtype=np.int64)
            p = o.compress(m)
            assert o.decompress(p).tolist() == m.tolist()


def pin_locality(o):
    """Fields are independent: a run of elements starting at a multiple of 64
    elements encodes to the corresponding bitstrings of the whole matrix."""
    rng = np.random.default_rng(3)
    for b in (1, 5, 10, 31, 33, 64):
        m = _random_matrix(rng, 9, 100, b, signed=(b > 32))
        p = o.compress(m)
        flat = m.reshape(-1)
        for start in (0, 64, 192, 576):
            n = min(128, flat.size - start)
            w = o.encode_run(flat[start:start + n], p.bits, nwords=(n * p.bits + 63) // 64)
            w0 = start * p.bits // 64
            full = p.payload[w0:w0 + w.size].copy()
            if (n * p.bits) % 64:
                full[-1] &= np.uint64((1 << ((n * p.bits) % 64)) - 1)
            assert np.array_equal(full, w), (b, start)
            back = o.decode_run(p.payload[w0:], n, p.bits, p.is_signed)
            assert np.array_equal(back, flat[start:start + n])


def pin_get(o):
    """get(i, j) equals the (i, j) element; out-of-range indices are rejected."""
    import oracle as _mod
    rng = np.random.default_rng(9)
    m = _random_matrix(rng, 6, 11, 13, True)
    p = o.compress(m)
    for i in range(6):
        for j in range(11):
            assert o.get(p, i, j) == m[i, j]
    for i, j in ((-1, 0), (6, 0), (0, 11), (0, -1)):
        try:
            o.get(p, i, j)
        except _mod.OracleError as e:
            assert e.code == _mod.E_RANGE
        else:
            raise AssertionError("out-of-range get accepted")


# ---------------------------------------------------------------------------
# operations: brute force on uncompressed values
# ---------------------------------------------------------------------------

def _py(m):
    return [[int(v) for v in row] for row in np.asarray(m)]


def _check_ops(o, A, B, x, s, C=None):
    pa, pb = o.compress(A), o.compress(B)
    a, b = _py(A), _py(B)
    rows, cols = len(a), len(a[0])
    add = [[a[i][j] + b[i][j] for j in range(cols)] for i in range(rows)]
    got = o.add(pa, pb)
    assert _py(o.decompress(got)) == add
    lo, hi = min(map(min, add)), max(map(max, add))
    assert (got.vmin, got.vmax) == (lo, hi) and (got.bits, got.is_signed) == _min_width(lo, hi)
    sc = [[s * a[i][j] for j in range(cols)] for i in range(rows)]
    got = o.scale(pa, s)
    assert _py(o.decompress(got)) == sc
    lo, hi = min(map(min, sc)), max(map(max, sc))
    assert (got.bits, got.is_signed) == _min_width(lo, hi)
    y = [_to_signed64(sum(a[i][j] * int(x[j]) for j in range(cols))) for i in range(rows)]
    assert o.matvec(pa, x).tolist() == y
    if C is not None:
        pc = o.compress(C)
        c = _py(C)
        mm = [[sum(a[i][k] * c[k][j] for k in range(cols)) for j in range(len(c[0]))]
              for i in range(rows)]
        got = o.matmul(pa, pc)
        assert _py(o.decompress(got)) == mm
        lo, hi = min(map(min, mm)), max(map(max, mm))
        assert (got.bits, got.is_signed) == _min_width(lo, hi)
        ii = [i for i in range(rows) for _ in range(len(c[0]))]
        jj = [j for _ in range(rows) for j in range(len(c[0]))]
        assert o.matmul_entries(pa, pc, ii, jj).tolist() == [mm[i][j] for i, j in zip(ii, jj)]


def pin_ops_bruteforce(o):
    """add, scale, matvec and matmul equal Python integer arithmetic on the values."""
    rng = np.random.default_rng(13)
    for trial in range(40):
        rows, cols, k2 = (int(v) for v in rng.integers(1, 9, size=3))
        ba, bb = (int(v) for v in rng.integers(1, 40, size=2))
        A = _random_matrix(rng, rows, cols, ba, bool(trial % 2))
        B = _random_matrix(rng, rows, cols, bb, bool(trial % 3 == 0))
        C = _random_matrix(rng, cols, k2, int(rng.integers(1, 20)), bool(trial % 5 == 0))
        x = rng.integers(-2**31, 2**31, size=cols, dtype=np.int64)
        s = int(rng.integers(-1000, 1000))
        _check_ops(o, A, B, x, s, C)
    # matvec wraps modulo 2^64
    A = np.full((2, 3), 2**62, dtype=np.int64)
    x = np.array([3, 5, 1], dtype=np.int64)  # exact row sum 9 * 2^62 = 2^65 + 2^62
    assert o.matvec(o.compress(A), x).tolist() == [2**62] * 2


def pin_ops_exhaustive_2x2(o):
    """Every 2x2 matrix of 2-bit unsigned values against every signed 2-bit partner."""
    una = list(itertools.product(range(4), repeat=4))
    sgn = list(itertools.product(range(-2, 2), repeat=4))
    x = np.array([3, -5], dtype=np.int64)
    partners = sgn[::17]
    for va in una:
        A = np.array(va, dtype=np.int64).reshape(2, 2)
        pa = o.compress(A)
        a = _py(A)
        assert o.matvec(pa, x).tolist() == [a[i][0] * 3 - a[i][1] * 5 for i in range(2)]
        for vb in partners:
            B = np.array(vb, dtype=np.int64).reshape(2, 2)
            pb = o.compress(B)
            b = _py(B)
            assert _py(o.decompress(o.add(pa, pb))) == [[a[i][j] + b[i][j] for j in range(2)]
                                                       for i in range(2)]
            assert _py(o.decompress(o.matmul(pa, pb))) == [
                [a[i][0] * b[0][j] + a[i][1] * b[1][j] for j in range(2)] for i in range(2)]
    for vb in sgn:
        B = np.array(vb, dtype=np.int64).reshape(2, 2)
        pb = o.compress(B)
        b = _py(B)
        assert _py(o.decompress(o.scale(pb, -3))) == [[-3 * v for v in row] for row in b]
        assert o.matvec(pb, x).tolist() == [b[i][0] * 3 - b[i][1] * 5 for i in range(2)]


def pin_identities(o):
    """A e_j = column j, A 1 = row sums, A + 0 = A, 1 A = A, 0 A = 0 (b = 1),
    A I = A, (A + B) x = A x + B x (mod 2^64)."""
    rng = np.random.default_rng(17)
    for b, signed in ((1, False), (10, False), (12, True), (31, True), (40, False)):
        A = _random_matrix(rng, 7, 9, b, signed)
        B = _random_matrix(rng, 7, 9, max(1, b - 3), not signed)
        pa, pb = o.compress(A), o.compress(B)
        for j in range(9):
            e = np.zeros(9, dtype=np.int64)
            e[j] = 1
            assert o.matvec(pa, e).tolist() == A[:, j].tolist()
        assert o.matvec(pa, np.ones(9, dtype=np.int64)).tolist() == [
            _to_signed64(sum(int(v) for v in row)) for row in A]
        zero = o.compress(np.zeros((7, 9), dtype=np.int64))
        same = o.add(pa, zero)
        assert (o.header(same), same.payload_bytes()) == (o.header(pa), pa.payload_bytes())
        one = o.scale(pa, 1)
        assert (o.header(one), one.payload_bytes()) == (o.header(pa), pa.payload_bytes())
        z = o.scale(pa, 0)
        assert z.bits == 1 and not z.is_signed and not z.payload.any()
        neg = o.scale(pa, -1)
        assert np.array_equal(o.decompress(neg), -A)
        assert neg.is_signed == (int(A.max()) > 0)
        eye = o.compress(np.eye(9, dtype=np.int64))
        ai = o.matmul(pa, eye)
        assert (o.header(ai), ai.payload_bytes()) == (o.header(pa), pa.payload_bytes())
        x = rng.integers(-2**31, 2**31, size=9, dtype=np.int64)
        lhs = o.matvec(o.add(pa, pb), x)
        rhs = [_to_signed64(int(u) + int(v)) for u, v in zip(o.matvec(pa, x), o.matvec(pb, x))]
        assert lhs.tolist() == rhs


def pin_overflow_rules(o):
    """add and scale fail exactly when a result leaves int64; matmul fails iff
    K * max|A| * max|B| >= 2^63; matvec never fails (it wraps)."""
    import oracle as _mod

    def raises(fn):
        try:
            fn()
        except _mod.OracleError as e:
            return e.code
        return None

    big = o.compress(np.array([[2**63 - 1, 0]], dtype=np.int64))
    one = o.compress(np.array([[1, 0]], dtype=np.int64))
    m1 = o.compress(np.array([[-1, 0]], dtype=np.int64))
    assert raises(lambda: o.add(big, one)) == _mod.E_OVERFLOW
    assert raises(lambda: o.add(big, m1)) is None
    low = o.compress(np.array([[-2**63, 1]], dtype=np.int64))
    assert raises(lambda: o.scale(low, -1)) == _mod.E_OVERFLOW
    assert raises(lambda: o.scale(low, 1)) is None
    assert raises(lambda: o.scale(o.compress(np.array([[2**32]], dtype=np.int64)), 2**31)) \
        == _mod.E_OVERFLOW
    assert raises(lambda: o.scale(o.compress(np.array([[2**31]], dtype=np.int64)), 2**31)) is None
    a1 = o.compress(np.array([[2**31]], dtype=np.int64))
    a2 = o.compress(np.array([[2**31, 2**31]], dtype=np.int64))
    bcol = o.compress(np.array([[2**31], [-2**31]], dtype=np.int64))
    b1 = o.compress(np.array([[-2**31]], dtype=np.int64))
    # K=2: bound 2 * 2^31 * 2^31 = 2^63 -> rejected even though the exact entry is 0
    assert raises(lambda: o.matmul(a2, bcol)) == _mod.E_OVERFLOW
    # K=1: bound 2^62 -> accepted
    assert o.decompress(o.matmul(a1, b1)).tolist() == [[-2**62]]
    assert raises(lambda: o.matmul(a1, a2)) is None  # 1x1 * 1x2
    assert raises(lambda: o.matmul(a2, a2)) == _mod.E_SHAPE
    assert raises(lambda: o.add(a1, a2)) == _mod.E_SHAPE


# ---------------------------------------------------------------------------
# Column-major unravel and y = A^T x
# ---------------------------------------------------------------------------

def pin_cm_worked_example(o):
    """A single row or a single column unravels the same way by row or by
    column: both give the worked example's bitstrings."""
    g = _golden_kv("sm_worked_example.txt")
    vals = [int(v) for v in g["values"].split()]
    want = [int(g["bitstring_1"].replace(" ", ""), 2), int(g["bitstring_2"].replace(" ", ""), 2)]
    for A in (np.array([vals]), np.array([vals]).T):
        p = o.compress_cm(A)
        assert [int(w) for w in p.payload] == want and p.bits == 10
        assert o.decompress_cm(p).tolist() == A.tolist()
    h = o.header_cm(o.compress_cm(np.array([vals]).T))
    assert h[7] == 2 and int.from_bytes(h[8:16], "little") == 8
    assert int.from_bytes(h[16:24], "little") == 1


def pin_cm_layout(o):
    """Column-major streams read back field by field: element (i, j) at stream
    index j*rows + i, same widths and word count as row-major."""
    rng = np.random.default_rng(31)
    for t in range(40):
        r, c = int(rng.integers(1, 20)), int(rng.integers(1, 20))
        b = int(rng.integers(1, 65))
        signed = b == 64 or t % 2 == 1
        A = _random_matrix(rng, r, c, b, signed)
        p = o.compress_cm(A)
        q = o.compress(A)
        assert (p.bits, p.is_signed, p.words) == (q.bits, q.is_signed, q.words)
        stream = sum(int(w) << (64 * k) for k, w in enumerate(p.payload))
        for i in range(r):
            for j in range(c):
                u = (stream >> ((j * r + i) * p.bits)) & ((1 << p.bits) - 1)
                assert u == int(A[i, j]) & ((1 << p.bits) - 1), (i, j)
        assert stream >> (r * c * p.bits) == 0
        assert o.decompress_cm(p).tolist() == A.tolist()
        i, j = int(rng.integers(0, r)), int(rng.integers(0, c))
        assert o.get_cm(p, i, j) == int(A[i, j])


def pin_transposed_products_bruteforce(o):
    """y = A x (column-major A) and y = A^T x (both layouts) against Python
    integers modulo 2^64, and the identity matvec_t(A, e_i) = row i of A."""
    rng = np.random.default_rng(37)
    for t in range(40):
        r, c = int(rng.integers(1, 30)), int(rng.integers(1, 30))
        b = [1, 5, 17, 33, 62][t % 5]
        A = _random_matrix(rng, r, c, b, t % 2 == 1)
        xr = rng.integers(-2**62, 2**62, size=r, dtype=np.int64)
        xc = rng.integers(-2**62, 2**62, size=c, dtype=np.int64)
        L = A.tolist()
        want_t = [_to_signed64(sum(L[i][j] * int(xr[i]) for i in range(r))) for j in range(c)]
        want = [_to_signed64(sum(L[i][j] * int(xc[j]) for j in range(c))) for i in range(r)]
        pr, pc = o.compress(A), o.compress_cm(A)
        assert o.matvec_t(pr, xr).tolist() == want_t
        assert o.matvec_t_cm(pc, xr).tolist() == want_t
        assert o.matvec_cm(pc, xc).tolist() == want
        i = int(rng.integers(0, r))
        e = np.zeros(r, dtype=np.int64)
        e[i] = 1
        assert o.matvec_t(pr, e).tolist() == L[i]


# ---------------------------------------------------------------------------
# Method 2 (Variable Length Blocks)
# ---------------------------------------------------------------------------

def _vlb_elem_width(v: int, signed: bool) -> int:
    """Fewest bits holding v alone: Eq. 1 on the element when unsigned; the
    smallest two's complement width, found by search, when signed."""
    if not signed:
        return max(1, v.bit_length())
    for b in range(1, 65):
        if -(1 << (b - 1)) <= v < (1 << (b - 1)):
            return b
    raise AssertionError(v)


def _vlb_read(payload, n: int, k: int, signed: bool):
    """Reads n (length, value) pairs from the bitstrings, least significant bit
    first, straddling freely; returns the values, the widths and the bits used."""
    stream = 0
    for i, w in enumerate(payload):
        stream |= int(w) << (64 * i)
    p, vals, widths = 0, [], []
    for _ in range(n):
        b = (stream >> p) & ((1 << k) - 1)
        p += k
        u = (stream >> p) & ((1 << b) - 1)
        p += b
        if signed and b and (u >> (b - 1)) & 1:
            u -= 1 << b
        vals.append(u)
        widths.append(b)
    return vals, widths, p, stream


def pin_vlb_worked_example(o):
    """Method 2's worked example: the states after steps 1-3 and the two final
    bitstrings, k = 4 and the 91 bits the printed layout uses."""
    g = _golden_kv("vlb_worked_example.txt")
    vals = [int(v) for v in g["values"].split()]
    w0 = int(g["bitstring_1"].replace(" ", ""), 2)
    w1 = int(g["bitstring_2"].replace(" ", ""), 2)
    p = o.vlb_compress(np.array([vals], dtype=np.int64))
    assert p.k == int(g["k"]) and not p.is_signed
    assert p.nbits == int(g["nbits"]) and p.words == int(g["words"])
    assert [int(w) for w in p.payload] == [w0, w1]
    for s in (1, 2, 3):
        q = o.vlb_compress(np.array([vals[:s]], dtype=np.int64))
        assert q.k == 4 and q.words == 1
        assert int(q.payload[0]) == int(g["step_%d" % s].replace(" ", ""), 2)
    assert o.vlb_decompress(p).tolist() == [vals]
    assert [o.vlb_get(p, 0, j) for j in range(8)] == vals
    # Eq. 16 with these frequencies: every element's k + b_i bits
    assert p.nbits == sum(4 + bl for _, _, bl in _table1())


def pin_vlb_layout(o):
    """Every stream read back by an independent sequential reader: the length
    chunk holds the element's minimal width, k = b(b(max)) (Eq. 16's k) for
    non-negative matrices, bits used = sum of k + b_i (Eq. 16), floor(bits/64)
    + 1 bitstrings with zero padding; signed matrices use minimal two's
    complement widths."""
    rng = np.random.default_rng(21)
    shapes = [(1, 1), (1, 7), (3, 5), (4, 33), (9, 64), (17, 31)]
    for t in range(60):
        r, c = shapes[t % len(shapes)]
        signed = t % 3 == 2
        top = int(rng.integers(1, 64))
        lens = rng.integers(0, top + 1, size=r * c)
        mag = np.array([int(rng.integers(0, 1 << int(L))) if L else 0 for L in lens],
                       dtype=np.uint64)
        v = mag.astype(np.int64)
        if signed:
            neg = rng.random(r * c) < 0.5
            v = np.where(neg, -v - 1, v)
        A = v.reshape(r, c)
        p = o.vlb_compress(A)
        flat = [int(e) for e in A.ravel()]
        is_signed = min(flat) < 0
        assert p.is_signed == is_signed
        widths = [_vlb_elem_width(e, is_signed) for e in flat]
        k = max(widths).bit_length()
        if not is_signed:
            assert k == max(1, max(flat).bit_length()).bit_length()
        assert p.k == k
        assert p.nbits == sum(k + b for b in widths)
        assert p.words == p.nbits // 64 + 1
        got, got_w, used, stream = _vlb_read(p.payload, r * c, k, is_signed)
        assert got == flat and got_w == widths and used == p.nbits
        assert stream >> p.nbits == 0
        assert o.vlb_decompress(p).tolist() == A.tolist()
        # element starts: prefix sums of k + b_e
        starts = np.concatenate([[0], np.cumsum([k + b for b in widths])[:-1]]).reshape(r, c)
        for grp in (1, 3, 32):
            assert o.vlb_offsets(p, grp).tolist() == starts[:, ::grp].tolist()


def pin_vlb_extremes(o):
    """The widest elements (64-bit, 7-bit length chunks) and the narrowest (all
    zeros: one bit each, k = 1)."""
    A = np.array([[-2**63, 2**63 - 1, 0, -1, 1]], dtype=np.int64)
    p = o.vlb_compress(A)
    assert p.is_signed and p.k == 7
    got, widths, used, _ = _vlb_read(p.payload, 5, 7, True)
    assert got == A.ravel().tolist() and widths == [64, 64, 1, 1, 2] and used == p.nbits
    z = o.vlb_compress(np.zeros((3, 70), dtype=np.int64))
    assert z.k == 1 and z.nbits == 3 * 70 * 2 and not z.is_signed
    # each element: length chunk "1", value "0"
    stream = sum(int(w) << (64 * i) for i, w in enumerate(z.payload))
    assert stream == sum(1 << (2 * e) for e in range(210))
    u = o.vlb_compress(np.array([[2**63 - 1, 1, 0]], dtype=np.int64))
    assert not u.is_signed and u.k == 6 and u.nbits == 3 * 6 + 63 + 1 + 1


def pin_vlb_ops_bruteforce(o):
    """get and matvec on Method 2 matrices against Python integers (mod 2^64)."""
    rng = np.random.default_rng(23)
    for t in range(30):
        r, c = int(rng.integers(1, 12)), int(rng.integers(1, 40))
        top = [3, 10, 20, 40, 62][t % 5]
        A = rng.integers(-(1 << top) if t % 2 else 0, 1 << top, size=(r, c), dtype=np.int64)
        x = rng.integers(-2**62, 2**62, size=c, dtype=np.int64)
        p = o.vlb_compress(A)
        want = [_to_signed64(sum(int(a) * int(b) for a, b in zip(row, x))) for row in A.tolist()]
        assert o.vlb_matvec(p, x).tolist() == want
        for _ in range(5):
            i, j = int(rng.integers(0, r)), int(rng.integers(0, c))
            assert o.vlb_get(p, i, j) == int(A[i, j])


def pin_vlb_exhaustive_small(o):
    """Every 1 x 3 matrix with entries in [-4, 7]: stream read back exactly."""
    for vals in itertools.product(range(-4, 8), repeat=3):
        A = np.array([vals], dtype=np.int64)
        p = o.vlb_compress(A)
        signed = min(vals) < 0
        widths = [_vlb_elem_width(v, signed) for v in vals]
        k = max(widths).bit_length()
        got, got_w, used, stream = _vlb_read(p.payload, 3, k, signed)
        assert (p.k, p.nbits) == (k, used)
        assert got == list(vals) and got_w == widths and stream >> used == 0


# ---------------------------------------------------------------------------
# Choosing the method (Eq. 14-17, 29; Discussion)
# ---------------------------------------------------------------------------

def _efficiency_table():
    rows = []
    with open(os.path.join(GOLDEN, "efficiency_tables.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _of_length(L: int) -> int:
    """A value whose two's complement width is exactly L (a signed matrix:
    bit-lengths up to 64 need the sign reading)."""
    return -(1 << (L - 1))


def pin_method_worked_example(o):
    """The worked example: 80 bits with Method 1, 91 with Method 2 (as the
    printed bitstrings lay out), so Method 1; eta_1 = (64 - 10)/64 (Eq. 15)."""
    info = o.method_info(np.array([[900, 1023, 721, 256, 1, 10, 700, 20]]))
    assert (info["sm_bits"], info["sm_nbits"], info["vlb_k"], info["vlb_nbits"]) == (10, 80, 4, 91)
    assert info["method"] == 1 and info["eta1"] == 54 / 64 and info["eta2"] == 1 - 91 / 512


def pin_method_paper_values(o):
    """Eq. 17 on matrices built to the Discussion's bit-length mixes: Table 2,
    the equal-group examples and the half-1/half-64 example, to the printed
    digits; every one of them picks Method 2 (eta_1 = 0 at width 64)."""
    for row in _efficiency_table():
        kind = row[0]
        # Table 2 and the group list print eta_2 truncated (not rounded) to 3
        # and 4 decimals; the half-and-half example rounds intermediate terms.
        if kind == "two_groups":
            p1, want, digits = float(row[1]), float(row[2]), 3
            n1 = round(10 * p1)
            vals = [0] * n1 + [_of_length(64)] * (10 - n1)
        elif kind == "groups":
            vals = [_of_length(int(L)) if int(L) > 1 else 0 for L in row[1].split(",")]
            want, digits = float(row[2]), 4
        elif kind == "half_1_64":
            vals = [0, _of_length(64)] * 4
            want, digits = float(row[1]), None
        else:
            continue
        info = o.method_info(np.array([vals], dtype=np.int64))
        assert info["vlb_k"] == 7 and info["sm_bits"] == 64 and info["eta1"] == 0.0
        n = len(vals)
        exact = Fraction(64 * n - info["vlb_nbits"], 64 * n)  # Eq. 14 with Eq. 16's bits
        assert abs(info["eta2"] - float(exact)) < 1e-15
        if digits is None:
            assert abs(exact - Fraction(row[1])) <= Fraction(1, 10 ** 4), (row, exact)
        else:
            assert math.trunc(exact * 10 ** digits) == round(want * 10 ** digits), (row, exact)
        assert info["method"] == (2 if info["vlb_nbits"] < info["sm_nbits"] else 1)


def pin_eta2_model_tables(o):
    """Eq. 29 with k = 7 against Tables 3-5 (uniform, binomial, truncated
    Poisson bit-lengths) and Eq. 45 (38.28 %)."""
    from math import comb, exp, lgamma, log
    for row in _efficiency_table():
        kind, par, want = row[0], int(row[1]) if row[0] in ("uniform", "binomial", "poisson") \
            else None, float(row[-1])
        if kind == "uniform":
            pmf = [1.0 / par if b <= par else 0.0 for b in range(1, 65)]
        elif kind == "binomial":
            # the first column is n (Table 4's caption; its header says n p):
            # the printed values fit E(B) = n / 2
            n = par
            pmf = [comb(n, b) / 2.0 ** n if b <= n else 0.0 for b in range(1, 65)]
        elif kind == "poisson":
            pmf = [exp(b * log(par) - par - lgamma(b + 1)) for b in range(1, 65)]
        else:
            continue
        assert abs(o.eta2_model(pmf, 7) - want) <= 1e-4, (row, o.eta2_model(pmf, 7))
    assert round(100 * o.eta2_model([1 / 64] * 64, 7), 2) == 38.28
    # the model equals the exact eta_2 of a matrix with that bit-length mix
    vals = [_of_length(L) if L > 1 else 0 for L in range(1, 65)]
    info = o.method_info(np.array([vals], dtype=np.int64))
    assert abs(info["eta2"] - o.eta2_model([1 / 64] * 64, 7)) < 1e-12


def pin_method_bruteforce(o):
    """Bit counts against brute force; Method 2 iff it uses strictly fewer
    bits; a tie (here 32 bits each) goes to Method 1."""
    rng = np.random.default_rng(41)
    for t in range(60):
        r, c = int(rng.integers(1, 12)), int(rng.integers(1, 12))
        top = int(rng.integers(1, 63))
        A = rng.integers(0, 1 << top, size=(r, c), dtype=np.int64) >> rng.integers(0, top + 1,
                                                                                   size=(r, c))
        if t % 3 == 0:
            A = -A - 1 + (A % 2)
        flat = [int(v) for v in A.ravel()]
        signed = min(flat) < 0
        b = _min_width(min(flat), max(flat))[0]
        widths = [_vlb_elem_width(v, signed) for v in flat]
        k = max(widths).bit_length()
        info = o.method_info(A)
        assert info["sm_bits"] == b and info["sm_nbits"] == r * c * b
        assert info["vlb_k"] == k and info["vlb_nbits"] == sum(k + w for w in widths)
        assert info["method"] == (2 if sum(k + w for w in widths) < r * c * b else 1)
    tie = o.method_info(np.array([[1 << 15, 1 << 5]]))
    assert tie["sm_nbits"] == tie["vlb_nbits"] == 32 and tie["method"] == 1


# ---- floats in fixed point (Conclusion) ------------------------------------

def _rne_fraction(x: Fraction) -> int:
    """Round half to even of an exact rational (Python's round on Fraction)."""
    return round(x)


def _fx_cases(rng):
    """(values as float64, f) cases: random magnitudes over the exponent
    range, exact ties, subnormals, zeros of both signs."""
    cases = []
    for f in (0, 1, 7, 20, 52, -3, -40, 300, 1074):
        # |v * 2^f| < 2^61: v = m * 2^(k - f) with |m| < 2^53, k <= 8
        m = rng.integers(-(1 << 53) + 1, 1 << 53, size=40)
        k = rng.integers(-60, 9, size=40)
        v = np.array([math.ldexp(float(mi), int(ki) - f) for mi, ki in zip(m, k)])
        t = rng.integers(-(1 << 40), 1 << 40, size=10)
        ties = np.array([math.ldexp(float(ti) + 0.5, -f) for ti in t])
        cases.append((np.concatenate([v, ties, [0.0, -0.0, math.ldexp(1.0, -f - 2),
                                                 -math.ldexp(3.0, -f - 1)]]), f))
    sub = np.array([5e-324, -5e-324, 2.5e-320, math.ldexp(1.0, -1074) * 7])
    cases.append((sub, 1074))
    cases.append((sub, 1076))
    return cases


def pin_fixed_point_quantize(o):
    """q = round-half-to-even(v * 2^f) against exact rational arithmetic, for
    float64 and float32 inputs, including ties (to even), subnormals and
    signed zeros; the rounding error is at most 2^-(f+1)."""
    rng = np.random.default_rng(53)
    for v, f in _fx_cases(rng):
        want = [_rne_fraction(Fraction(float(x)) * Fraction(2) ** f) for x in v]
        assert o.quantize(v, f).tolist() == want, f
        for x, q in zip(v, want):
            assert abs(Fraction(float(x)) - Fraction(q) / Fraction(2) ** f) <= \
                Fraction(1, 2) / Fraction(2) ** f
        v32 = v.astype(np.float32)
        want32 = [_rne_fraction(Fraction(float(x)) * Fraction(2) ** f) for x in v32]
        assert o.quantize(v32, f).tolist() == want32, f
    # every half-integer multiple of 2^-f goes to the even neighbour
    halves = np.array([k + 0.5 for k in range(-6, 6)])
    assert o.quantize(halves, 0).tolist() == [-6, -4, -4, -2, -2, 0, 0, 2, 2, 4, 4, 6]


def pin_fixed_point_errors(o):
    """NaN and infinities are out of range (wherever they are, before any
    overflow); |v * 2^f| >= 2^62 overflows, the largest double below it does
    not."""
    import oracle
    for bad in (math.nan, math.inf, -math.inf):
        try:
            o.quantize(np.array([1.0, math.ldexp(1.0, 70), bad]), 3)
            raise AssertionError("NaN / infinity accepted")
        except oracle.OracleError as e:
            assert e.code == oracle.E_RANGE
    for f in (0, 10, -10):
        edge = math.ldexp(1.0, 62 - f)
        for v in (edge, -edge, math.ldexp(1.0, 1023)):
            try:
                o.quantize(np.array([v]), f)
                raise AssertionError("overflow accepted")
            except oracle.OracleError as e:
                assert e.code == oracle.E_OVERFLOW
        below = math.nextafter(edge, 0.0)
        assert o.quantize(np.array([below, -below]), f).tolist() == [(1 << 62) - 512,
                                                                      -(1 << 62) + 512]


def pin_fixed_point_dequantize(o):
    """v = q 2^-f: q rounded to double (half to even), then scaled (rounded
    once if subnormal), against exact rationals; float32 rounds that double
    once more."""
    rng = np.random.default_rng(59)
    q = np.concatenate([rng.integers(-(1 << 62), 1 << 62, size=40),
                        rng.integers(-(1 << 20), 1 << 20, size=40),
                        [0, 1, -1, (1 << 53) + 1, (1 << 62) - 1, -(1 << 62)]]).astype(np.int64)
    for f in (0, 3, 40, -5, 1074, 1100, 1200):
        got = o.dequantize(q, f)
        want = [float(Fraction(float(int(x))) / Fraction(2) ** f) for x in q]
        assert got.view(np.uint64).tolist() == np.array(want).view(np.uint64).tolist(), f
        got32 = o.dequantize(q, f, np.float32)
        assert got32.view(np.uint32).tolist() == \
            np.array(want).astype(np.float32).view(np.uint32).tolist(), f


def pin_fixed_point_frac_bits(o):
    """f = p - 1 - floor(log2 max|v|), so that 2^(p-1) <= max|v| 2^f < 2^p;
    the width of the quantized matrix is then p to p + 2 bits."""
    import oracle
    table = [(1.0, 10, 9), (0.75, 10, 10), (1000.0, 10, 0), (1023.999, 10, 0),
             (1024.0, 10, -1), (0.0, 7, 0), (5e-324, 1, 1074), (5e-324, 62, 1135),
             (1.7976931348623157e308, 62, -962), (0.5, 1, 1)]
    for a, p, f in table:
        assert o.frac_bits(a, p) == f, (a, p)
    for a, p in ((1.0, 0), (1.0, 63), (-1.0, 5), (math.nan, 5), (math.inf, 5)):
        try:
            o.frac_bits(a, p)
            raise AssertionError("invalid frac_bits arguments accepted")
        except oracle.OracleError as e:
            assert e.code == oracle.E_INVAL
    rng = np.random.default_rng(61)
    for _ in range(60):
        p = int(rng.integers(1, 40))
        v = rng.standard_normal(size=(3, 5)) * 10.0 ** rng.integers(-30, 30)
        a = float(np.abs(v).max())
        f = o.frac_bits(a, p)
        s = Fraction(a) * Fraction(2) ** f
        assert Fraction(2) ** (p - 1) <= s < Fraction(2) ** p
        qm = o.quantize(v, f)
        b = o.compress(qm).bits
        assert p <= b <= p + 2, (p, b)


def pin_fixed_point_headers(o):
    """Fixed-point matrices against headers and bitstrings derived by hand:
    the quantized values, flags bit 2, f at bytes 48..49 (positive and
    negative f), and a tie rounded to even."""
    g = _golden_kv("fixed_point_headers.txt")
    hx = lambda key: bytes(int(t, 16) for t in g[key].split())
    mat = lambda key, ty: np.array([[ty(v) for v in r.split()] for r in g[key].split(";")])
    for c in ("a", "b"):
        f = int(g[c + "_frac_bits"])
        q = o.quantize(mat(c + "_values", float), f)
        assert q.tolist() == mat(c + "_q", int).tolist()
        p = o.compress(q)
        assert p.bits == int(g[c + "_bits"])
        assert o.header_fx(p, f) == hx(c + "_header")
        assert [int(w) for w in p.payload] == [int(g[c + "_payload"], 16)]
        assert o.dequantize(o.decompress(p), f).tolist() == mat(c + "_values", float).tolist() \
            or c == "b"


ALL_PINS = [pin_table1, pin_eq1_special_case, pin_bitlen_bruteforce, pin_width_bruteforce,
            pin_worked_example, pin_signed_headers, pin_word_count, pin_round_trip, pin_signed_small_bruteforce,
            pin_locality, pin_get, pin_ops_bruteforce, pin_ops_exhaustive_2x2, pin_identities,
            pin_overflow_rules, pin_vlb_worked_example, pin_vlb_layout, pin_vlb_extremes,
            pin_vlb_ops_bruteforce, pin_vlb_exhaustive_small, pin_cm_worked_example,
            pin_cm_layout, pin_transposed_products_bruteforce, pin_method_worked_example,
            pin_method_paper_values, pin_eta2_model_tables, pin_method_bruteforce,
            pin_fixed_point_quantize, pin_fixed_point_errors, pin_fixed_point_dequantize,
            pin_fixed_point_frac_bits, pin_fixed_point_headers]
