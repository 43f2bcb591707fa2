"""A matrix of more than 2^32 elements (65537 x 65536 at one bit, 537 MB
packed, generated on the device): element, stream-word and row offsets past
32 bits in get, gather, matvec, y = A^T x, add and scale, checked on sampled
entries, rows and columns regenerated on the host against the oracle."""
import numpy as np
import pytest

import ccm_workloads as W
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROWS, COLS = 65537, 65536  # ROWS * COLS = 2^32 + 2^16


@pytest.fixture(scope="module")
def big():
    assert torch.cuda.is_available(), "gpu tests need a GPU"
    import paper_1303_0270_amd as c
    spec = W.MatrixSpec(ROWS, COLS, 0, 2, W.seed_for(9, 0), 3)
    A = c.generate(ROWS, COLS, spec.lo, spec.hi, spec.seed, spec.stream)
    assert (A.bits, A.is_signed, A.vmin, A.vmax) == (1, False, 0, 1)
    yield c, spec, A
    del A
    torch.cuda.empty_cache()


def far_indices(rng):
    e = [0, 2**32 - 1, 2**32, 2**32 + 1, ROWS * COLS - 1]
    e += [int(v) for v in rng.integers(2**32 - 2**20, ROWS * COLS, 11)]
    return np.array(e, dtype=np.int64)


def test_get_and_gather_past_2_32(big):
    c, spec, A = big
    e = far_indices(np.random.default_rng(1))
    want = W.uniform_at(spec.seed, spec.stream, e, spec.lo, spec.hi)
    ii, jj = e // COLS, e % COLS
    for k in (0, 1, 2, 4, len(e) - 1):
        assert c.get(A, int(ii[k]), int(jj[k])) == int(want[k])
    vals, bad = c.gather(A, torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda())
    assert not bad and np.array_equal(vals.cpu().numpy(), want)


def test_matvec_rows_past_2_32(big):
    c, spec, A = big
    x = W.uniform(W.seed_for(9, 2), 0, 0, COLS, -(1 << 15), 1 << 15)
    y = c.matvec(A, torch.from_numpy(x).to(torch.int32).cuda()).cpu().numpy()
    for r in (0, 1, 32767, 65535, ROWS - 1):
        row = spec.rows_slice(r, r + 1)
        assert y[r] == oracle.matvec(oracle.compress(row), x)[0], r


def test_matvec_t_columns_past_2_32(big):
    c, spec, A = big
    x = W.uniform(W.seed_for(9, 2), 1, 0, ROWS, -(1 << 15), 1 << 15)
    y = c.matvec_t(A, torch.from_numpy(x).to(torch.int32).cuda()).cpu().numpy()
    for j in (0, 2047, 2048, 40000, COLS - 1):
        col = spec.column(j).reshape(-1, 1)
        assert y[j] == oracle.matvec_t(oracle.compress(col), x)[0], j


def test_add_and_scale_past_2_32(big):
    c, spec, A = big
    e = far_indices(np.random.default_rng(2))
    a = W.uniform_at(spec.seed, spec.stream, e, spec.lo, spec.hi)
    ii = torch.from_numpy(e // COLS).cuda()
    jj = torch.from_numpy(e % COLS).cuda()
    s = c.add(A, A)
    assert (s.bits, s.vmin, s.vmax) == (2, 0, 2)
    vals, bad = c.gather(s, ii, jj)
    assert not bad and np.array_equal(vals.cpu().numpy(), 2 * a)
    del s
    t = c.scale(A, -3)
    assert (t.bits, t.is_signed, t.vmin, t.vmax) == (3, True, -3, 0)
    vals, bad = c.gather(t, ii, jj)
    assert not bad and np.array_equal(vals.cpu().numpy(), -3 * a)
