"""Batched matvec (one persistent launch, optionally a HIP graph) against the
oracle and against the per-call path."""
import json

import numpy as np
import pytest

import ccm_workloads as W
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "gpu tests need a GPU"


def ccm():
    import paper_1303_0270_amd as c
    return c


def rand_matrix(rng, rows, cols, b, signed):
    lo, hi = ((-(1 << (b - 1)), (1 << (b - 1)) - 1) if signed else (0, (1 << b) - 1))
    m = rng.integers(lo, hi, size=(rows, cols), endpoint=True, dtype=np.int64)
    flat = m.reshape(-1)
    flat[int(rng.integers(0, flat.size))] = hi
    if signed:
        flat[int(rng.integers(0, flat.size))] = lo
    return m


def make_batch(rng, count, max_dim, widths):
    c = ccm()
    mats, packed, xs, xh = [], [], [], []
    for t in range(count):
        r, k = int(rng.integers(1, max_dim + 1)), int(rng.integers(1, max_dim + 1))
        b = int(widths[t % len(widths)])
        signed = bool(rng.integers(0, 2)) if b < 64 else True
        A = rand_matrix(rng, r, k, b, signed)
        mats.append(A)
        packed.append(c.compress(torch.from_numpy(A).cuda()))
        x = rng.integers(-(1 << 15), 1 << 15, size=k) if t % 3 else \
            rng.integers(-(1 << 31), 1 << 31, size=k)
        xh.append(x)
        xs.append(torch.from_numpy(x).to(torch.int32).cuda())
    return mats, packed, xs, xh


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_all_widths_matches_oracle(use_graph):
    c = ccm()
    rng = np.random.default_rng(41)
    mats, packed, xs, xh = make_batch(rng, 96, 300, list(range(1, 65)) + [1, 2, 3, 5, 12, 24])
    ys = [torch.full((m.rows,), -7, dtype=torch.int64, device="cuda") for m in packed]
    batch = c.Batch(packed)
    batch.set_io(xs, ys)
    batch.run(use_graph=use_graph)
    torch.cuda.synchronize()
    for A, m, x, y in zip(mats, packed, xh, ys):
        want = oracle.matvec(oracle.compress(A), x)
        assert np.array_equal(y.cpu().numpy(), want), (m.rows, m.cols, m.bits, m.is_signed)
    batch.close()


def test_graph_replays_follow_new_inputs():
    """Replays of the captured graph, with eager work and new x/y between them,
    each match the eager per-call results."""
    c = ccm()
    rng = np.random.default_rng(43)
    mats, packed, xs, xh = make_batch(rng, 40, 200, [1, 3, 7, 12, 17, 24, 31, 33])
    batch = c.Batch(packed)
    for rep in range(4):
        xs_r = [torch.from_numpy(rng.integers(-(1 << 15), 1 << 15, size=m.cols)).to(
            torch.int32).cuda() for m in packed]
        ys_r = [torch.empty(m.rows, dtype=torch.int64, device="cuda") for m in packed]
        batch.set_io(xs_r, ys_r)
        batch.run(use_graph=True)
        eager = [c.matvec(m, x) for m, x in zip(packed, xs_r)]
        torch.cuda.synchronize()
        for y, e in zip(ys_r, eager):
            assert torch.equal(y, e), rep
    assert batch.info()["items"] >= len(packed)
    batch.close()


def test_tuning_table_is_used(tmp_path):
    c = ccm()
    rng = np.random.default_rng(44)
    mats, packed, xs, xh = make_batch(rng, 6, 300, [5])
    table = tmp_path / "tune.json"
    table.write_text(json.dumps({"widths": {"5": {"tile_rows": 7, "rows_in_flight": 2}}}))
    b_default = c.Batch(packed)
    b_tuned = c.Batch(packed, tune_json=str(table))
    want_items = sum(-(-m.rows // 7) for m in packed)
    assert b_tuned.info()["items"] == want_items
    assert b_default.info()["items"] < want_items
    ys = [torch.empty(m.rows, dtype=torch.int64, device="cuda") for m in packed]
    b_tuned.set_io(xs, ys)
    b_tuned.run(use_graph=False)
    torch.cuda.synchronize()
    for A, x, y in zip(mats, xh, ys):
        assert np.array_equal(y.cpu().numpy(), oracle.matvec(oracle.compress(A), x))


@pytest.mark.parametrize("rif", [1, 2, 4])
@pytest.mark.parametrize("tile", [5, 100])
def test_rows_in_flight_and_ragged_items(tmp_path, rif, tile):
    """Every rows-in-flight setting (capped per width inside the kernel) with
    items shorter than a pass (rows past an item are read clamped and
    dropped) and longer ones."""
    c = ccm()
    rng = np.random.default_rng(50 + rif + tile)
    widths = [1, 2, 3, 4, 7, 8, 9, 12, 16, 17, 24, 31, 40]
    mats, packed, xs, xh = make_batch(rng, len(widths) * 2, 260, widths)
    table = tmp_path / "tune.json"
    table.write_text(json.dumps({"widths": {str(b): {"tile_rows": tile, "rows_in_flight": rif}
                                            for b in widths}}))
    batch = c.Batch(packed, tune_json=str(table))
    ys = [torch.full((m.rows,), 3, dtype=torch.int64, device="cuda") for m in packed]
    batch.set_io(xs, ys)
    batch.run(use_graph=True)
    torch.cuda.synchronize()
    for A, m, x, y in zip(mats, packed, xh, ys):
        want = oracle.matvec(oracle.compress(A), x)
        assert np.array_equal(y.cpu().numpy(), want), (m.rows, m.cols, m.bits, rif, tile)
    batch.close()


def test_batched_workload_matches_per_call_and_oracle():
    """The batched workload at full size (4096 matrices, 32..2048 x 32..2048,
    widths 1..24): every y equals the per-call path; 12 small sampled
    matrices are regenerated on the host and checked by the oracle."""
    c = ccm()
    items = W.batched()
    mats = [c.generate(it.a.rows, it.a.cols, it.a.lo, it.a.hi, it.a.seed, it.a.stream)
            for it in items]
    xs = []
    for it in items:
        x = torch.empty(it.x.n, dtype=torch.int32, device="cuda")
        c.fill_uniform(x, it.x.lo, it.x.hi, it.x.seed, it.x.stream)
        xs.append(x)
    ys = [torch.empty(m.rows, dtype=torch.int64, device="cuda") for m in mats]
    batch = c.Batch(mats)
    batch.set_io(xs, ys)
    batch.run(use_graph=True)
    torch.cuda.synchronize()
    for m, x, y in zip(mats, xs, ys):
        assert torch.equal(y, c.matvec(m, x))
    small = sorted(range(len(items)), key=lambda t: items[t].a.rows * items[t].a.cols)[:12]
    for t in small:
        A = items[t].a.dense()
        assert mats[t].bits == oracle.width(int(A.min()), int(A.max()))[0]
        assert np.array_equal(ys[t].cpu().numpy(),
                              oracle.matvec(oracle.compress(A), items[t].x.dense()))
    batch.close()
