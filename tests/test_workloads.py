"""The seeded input generator (no method arithmetic): SplitMix64 against its
published reference outputs, the range map, and the workload shapes."""
import numpy as np

import ccm_workloads as W


def test_splitmix64_reference_outputs():
    # first five outputs of SplitMix64 started from seed 1234567 (the reference
    # implementation's published example sequence)
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert W.splitmix64(1234567, np.arange(5, dtype=np.uint64)).tolist() == want


def test_uniform_range_and_determinism():
    for lo, hi in ((0, 2), (-8, 8), (0, 1 << 31), (-(1 << 15), 1 << 15), (5, 6), (0, 1 << 32)):
        v = W.uniform(99, 3, 10, 20000, lo, hi)
        assert v.min() >= lo and v.max() < hi
        assert np.array_equal(v, W.uniform(99, 3, 10, 20000, lo, hi))
        # a window of the stream equals the matching slice of a longer draw
        assert np.array_equal(W.uniform(99, 3, 110, 50, lo, hi), v[100:150])
    # power-of-two spans use the top bits: every value appears for small spans
    assert set(W.uniform(7, 0, 0, 4000, 0, 8).tolist()) == set(range(8))


def test_workload_shapes():
    a, b, x, s = W.small_plain()
    assert (a.rows, a.cols, a.lo, a.hi, x.hi, s) == (256, 256, 0, 1024, 1000, 7)
    a, b, x, s = W.sweep(12, True, 64)
    assert (a.lo, a.hi, x.lo, x.hi) == (-2048, 2048, -32768, 32768)
    items = W.batched(count=64)
    assert all(32 <= it.a.rows <= 2048 and 32 <= it.a.cols <= 2048 and 1 <= it.bits <= 24
               for it in items)
    pool = W.serving_pool(5e7, max_elems=1e6)
    assert all(1 <= p.bits <= 20 and p.rows * p.cols >= 1 for p in pool)
    total = sum(64 + 8 * ((p.rows * p.cols * p.bits) // 64 + 1) for p in pool)
    assert total >= 5e7


def test_column_and_uniform_at_match_the_dense_matrix():
    spec = W.MatrixSpec(37, 53, -9, 40, W.seed_for(2, 0), 5)
    A = spec.dense()
    for j in (0, 1, 52, 17):
        assert np.array_equal(spec.column(j), A[:, j])
    idx = np.array([0, 5, 1960, 37 * 53 - 1])
    assert np.array_equal(W.uniform_at(spec.seed, spec.stream, idx, spec.lo, spec.hi),
                          A.reshape(-1)[idx])
