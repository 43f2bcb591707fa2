"""Results whose width stays on the device (ccm_add_async, ccm_matmul_async):
the same header and payload bytes as the oracle (and as the blocking calls),
with every step enqueued and no host wait; several in flight at once on
different streams; device-found overflow reported in the result."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "gpu tests need a GPU"


def ccm():
    import paper_1303_0270_amd as c
    return c


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.int64).cuda()


def rand_matrix(rng, rows, cols, b, signed):
    lo, hi = ((-(1 << (b - 1)), (1 << (b - 1)) - 1) if signed else (0, (1 << b) - 1))
    m = rng.integers(lo, hi, size=(rows, cols), endpoint=True, dtype=np.int64)
    m.flat[int(rng.integers(0, m.size))] = hi
    if signed:
        m.flat[int(rng.integers(0, m.size))] = lo
    return m


def assert_same_packed(gpu, ref):
    assert gpu.header() == oracle.header(ref)
    assert gpu.payload_bytes() == ref.payload_bytes()
    assert not gpu.payload[8 * gpu.words:].cpu().numpy().any()


ADD_CASES = {
    # the headers' bound is the exact range: one pass
    "tight": lambda r, n: (r.integers(-2**14, 2**14, n), r.integers(-2**14, 2**14, n)),
    # bound [0, 2000], exact [0, 1000]: the device repacks at 10 bits
    "loose": lambda r, n: (np.where(np.arange(n) == 0, 1000, r.integers(0, 500, n)),
                           np.where(np.arange(n) == n - 1, 1000, r.integers(0, 500, n))),
    # bound signed, exact unsigned and narrower
    "sign_changes": lambda r, n: (np.where(np.arange(n) == 0, -5, r.integers(0, 91, n)),
                                  np.where(np.arange(n) == 0, 5, r.integers(0, 11, n))),
    # unsigned 32-bit class
    "u32": lambda r, n: (r.integers(0, 2**31 + 1, n), r.integers(0, 2**31, n)),
    # int64 class, bound loose
    "i64_loose": lambda r, n: (np.where(np.arange(n) == 0, 2**40, r.integers(0, 2**39, n)),
                               np.where(np.arange(n) == n - 1, 2**40, r.integers(0, 2**39, n))),
    # a 64-bit result
    "i64_full": lambda r, n: (r.integers(-2**62, 2**62, n), r.integers(-2**61, 2**61, n)),
    # a bound past int64 whose sums fit: range pass first, width on the device
    "bound_past_int64": lambda r, n: (np.where(np.arange(n) % 2 == 0, 2**62 + 7, -(2**62)),
                                      np.where(np.arange(n) % 2 == 0, -(2**62), 2**62 + 5)),
}


@pytest.mark.parametrize("case", sorted(ADD_CASES))
@pytest.mark.parametrize("shape", [(1, 1), (3, 37), (300, 1001)], ids=str)
def test_add_async_matches_oracle(case, shape):
    c = ccm()
    n = shape[0] * shape[1]
    rng = np.random.default_rng(len(case) * 13 + n)
    a, b = ADD_CASES[case](rng, n)
    A = np.asarray(a, dtype=np.int64).reshape(shape)
    B = np.asarray(b, dtype=np.int64).reshape(shape)
    ref = oracle.add(oracle.compress(A), oracle.compress(B))
    ga, gb = c.compress(dev(A)), c.compress(dev(B))
    p = c.add_async(ga, gb)
    assert_same_packed(p.get(), ref)
    assert p.done()


def test_add_async_overflow_on_device():
    """Sums past int64 (the bound leaves int64, so the device's range pass
    decides): the result reports CCM_E_OVERFLOW."""
    c = ccm()
    a = c.compress(dev(np.array([[2**63 - 1, 0]])))
    one = c.compress(dev(np.array([[1, 0]])))
    p = c.add_async(a, one)
    with pytest.raises(c.CcmError) as ei:
        p.get()
    assert ei.value.status == c._lib.E_OVERFLOW


MATMUL_CASES = [(10, False, 10, False), (6, False, 4, True), (1, False, 1, True),
                (20, True, 17, False), (8, False, 8, True), (2, True, 5, True)]


@pytest.mark.parametrize("ba,sa,bb,sb", MATMUL_CASES)
def test_matmul_async_matches_oracle_and_blocking(ba, sa, bb, sb):
    c = ccm()
    rng = np.random.default_rng(ba * 31 + bb)
    for M, K, N in ((1, 1, 1), (65, 33, 70), (257, 300, 131), (300, 200, 520)):
        A = rand_matrix(rng, M, K, ba, sa)
        B = rand_matrix(rng, K, N, bb, sb)
        ref = oracle.matmul(oracle.compress(A), oracle.compress(B))
        ga, gb = c.compress(dev(A)), c.compress(dev(B))
        got = c.matmul_async(ga, gb).get()
        assert_same_packed(got, ref)
        blocking = c.matmul(ga, gb)
        assert got.header() == blocking.header()
        assert got.payload_bytes() == blocking.payload_bytes()


def test_many_in_flight_on_streams():
    """Twelve results enqueued on three streams before any is read back, each
    with its own workspace; every one equals the oracle."""
    c = ccm()
    rng = np.random.default_rng(77)
    streams = [torch.cuda.Stream() for _ in range(3)]
    jobs = []
    for t in range(12):
        M, K, N = int(rng.integers(20, 200)), int(rng.integers(20, 300)), int(rng.integers(2, 65))
        A = rand_matrix(rng, M, K, int(rng.integers(1, 12)), False)
        B = rand_matrix(rng, K, N, int(rng.integers(1, 9)), True)
        X = rand_matrix(rng, M, K, int(rng.integers(1, 12)), bool(t % 2))
        ga, gb, gx = c.compress(dev(A)), c.compress(dev(B)), c.compress(dev(X))
        torch.cuda.synchronize()
        s = streams[t % 3]
        with torch.cuda.stream(s):
            pm = c.matmul_async(ga, gb, stream=s)
            pa = c.add_async(ga, gx, stream=s)
        jobs.append((pm, oracle.matmul(oracle.compress(A), oracle.compress(B))))
        jobs.append((pa, oracle.add(oracle.compress(A), oracle.compress(X))))
    for p, ref in jobs:
        assert_same_packed(p.get(), ref)
