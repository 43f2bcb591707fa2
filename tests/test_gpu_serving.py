"""Serving loop: every request's result in the mix equals the same request
run alone (bit for bit), sampled requests equal the oracle, launches overlap
on the device (matmuls beside matvecs), and admission holds requests back
when slots or memory run out."""
import numpy as np
import pytest

import ccm_workloads as W
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "gpu tests need a GPU"


# Matrices wider than the batched kernel's x staging (more than 8192
# columns): a served matvec launch runs them with the single-matrix kernel.
WIDE = [(1500, 20000, 7), (300, 9000, 13), (40, 65536, 2)]


def wide_specs(first_stream=9000):
    return [W.PoolMatrix(r, c, b, W.MatrixSpec(r, c, 0, 1 << b, W.seed_for(5, 1), first_stream + t))
            for t, (r, c, b) in enumerate(WIDE)]


@pytest.fixture(scope="module")
def pool():
    from paper_1303_0270_amd import serve
    specs = W.serving_pool(48e6, max_elems=2e6) + wide_specs()
    return specs, serve.make_pool(specs)


def mv_requests(pool_mats, mats, seed, first_rid, t_end):
    """One matvec request on each of `mats`, arrivals spread over [0, t_end)."""
    import paper_1303_0270_amd as c
    from paper_1303_0270_amd import serve
    out = []
    for k, mi in enumerate(mats):
        rid = first_rid + k
        x = torch.empty(pool_mats[mi].cols, dtype=torch.int32, device="cuda")
        c.fill_uniform(x, -(1 << 15), 1 << 15, seed, serve.X_STREAM + rid)
        out.append(serve.Request(rid, "mv", mi, t_end * k / max(1, len(mats)), x=x))
    torch.cuda.synchronize()
    return out


def sampled_rows(m, rows):
    rows = sorted(set(r for r in rows if 0 <= r < m.rows))
    return rows


def check_alone(c, pool_mats, reqs):
    for r in reqs:
        a = pool_mats[r.mat]
        if r.kind == "mv":
            assert torch.equal(r.y, c.matvec(a, r.x)), r.rid
        else:
            alone = c.matmul(a, r.b)
            assert r.c.header() == alone.header() and \
                r.c.payload_bytes() == alone.payload_bytes(), r.rid


def check_oracle_rows(specs, pool_mats, reqs, seed):
    """Matvec requests: sampled rows (first, last, two inside) against the
    oracle, each row encoded on its own at the matrix's width."""
    from paper_1303_0270_amd import serve
    for r in reqs:
        if r.kind != "mv":
            continue
        spec, a = specs[r.mat].spec, pool_mats[r.mat]
        x = W.uniform(seed, serve.X_STREAM + r.rid, 0, a.cols, -(1 << 15), 1 << 15)
        y = r.y.cpu().numpy()
        for row in sampled_rows(a, [0, a.rows - 1, a.rows // 3, (7 * a.rows) // 11]):
            vals = spec.rows_slice(row, row + 1)
            p = oracle.Packed(1, a.cols, int(vals.min()), int(vals.max()), a.bits,
                              a.is_signed, oracle.encode_run(vals, a.bits))
            assert y[row] == oracle.matvec(p, x)[0], (r.rid, row)


def check_oracle_full(specs, pool_mats, reqs, seed, count=8):
    from paper_1303_0270_amd import serve
    mv = [r for r in reqs if r.kind == "mv"]
    mv = sorted(mv, key=lambda r: pool_mats[r.mat].rows * pool_mats[r.mat].cols)[:count]
    for r in mv:
        A = specs[r.mat].spec.dense()
        x = W.uniform(seed, serve.X_STREAM + r.rid, 0, A.shape[1], -(1 << 15), 1 << 15)
        assert np.array_equal(r.y.cpu().numpy(), oracle.matvec(oracle.compress(A), x))
    mm = [r for r in reqs if r.kind == "mm"][:3]
    for r in mm:
        A = specs[r.mat].spec.dense()
        Bv = r.b
        lo, hi = (-(1 << (Bv.bits - 1)), 1 << (Bv.bits - 1)) if Bv.bits > 1 else (-1, 1)
        Bd = W.uniform_matrix(seed, serve.B_STREAM + r.rid, Bv.rows, Bv.cols, lo, hi)
        ref = oracle.matmul(oracle.compress(A), oracle.compress(Bd))
        assert r.c.header() == oracle.header(ref) and r.c.payload_bytes() == ref.payload_bytes()


@pytest.mark.parametrize("qps", [None, 30000.0])
def test_results_same_alone_and_in_mix(pool, qps):
    import paper_1303_0270_amd as c
    from paper_1303_0270_amd import serve
    specs, mats = pool
    seed = W.seed_for(5, 3)
    reqs = serve.make_requests(mats, 300, qps, seed, mm_frac=0.15)
    nwide = len(WIDE)
    wide_idx = list(range(len(mats) - nwide, len(mats)))
    t_end = max(r.arrival for r in reqs)
    reqs += mv_requests(mats, wide_idx * 2, seed, 5000, t_end)
    srv = serve.Server(mats, arena_bytes=1 << 30, streams=3, max_inflight=64, max_batch=32)
    stats = srv.run(reqs)
    srv.close()
    n = len(reqs)
    assert stats["requests"] == n and all(np.isfinite(r.done) for r in reqs)
    assert stats["launches"] < n or qps  # burst arrivals are batched
    assert all(r.done >= r.arrival - 1e-4 for r in reqs)
    # launches ran side by side on the device, matmuls beside matvecs
    assert stats["max_launches_in_flight"] >= 2
    assert stats["overlapped_launches"] >= 1
    if qps is None:
        assert stats["mm_overlapping_mv"] >= 1
    check_alone(c, mats, reqs)
    check_oracle_full(specs, mats, reqs, seed)
    check_oracle_rows(specs, mats, [r for r in reqs if r.mat in wide_idx], seed)


def test_requests_from_the_full_size_pool():
    """A handful of matrices drawn from the full 200 GB pool distribution
    (the largest about 10^9 elements), served in a mix of matvecs and
    matmuls; sampled rows of every matvec equal the oracle's and every result
    equals the same request run alone."""
    import paper_1303_0270_amd as c
    from paper_1303_0270_amd import serve
    full = W.serving_pool(200e9)
    sizes = np.array([p.rows * p.cols for p in full])
    rng = np.random.default_rng(W.seed_for(5, 6))
    picks = [int(np.argmax(sizes))] + [int(i) for i in rng.choice(len(full), 5, replace=False)]
    picks += [int(i) for i in np.flatnonzero(sizes <= 1 << 20)[:2]]  # matmul-sized
    specs = [full[i] for i in picks]
    mats = serve.make_pool(specs)
    seed = W.seed_for(5, 7)
    reqs = serve.make_requests(mats, 60, None, seed, mm_frac=0.2)
    reqs += mv_requests(mats, [0, 0], seed, 6000, 0.0)  # the largest matrix, twice
    srv = serve.Server(mats, arena_bytes=8 << 30, streams=4, max_inflight=64, max_batch=32)
    stats = srv.run(reqs)
    srv.close()
    assert stats["requests"] == len(reqs)
    check_alone(c, mats, reqs)
    check_oracle_rows(specs, mats, reqs, seed)
    mm = [r for r in reqs if r.kind == "mm"][:2]
    for r in mm:
        A = specs[r.mat].spec.dense()
        Bv = r.b
        lo, hi = (-(1 << (Bv.bits - 1)), 1 << (Bv.bits - 1)) if Bv.bits > 1 else (-1, 1)
        Bd = W.uniform_matrix(seed, serve.B_STREAM + r.rid, Bv.rows, Bv.cols, lo, hi)
        ref = oracle.matmul(oracle.compress(A), oracle.compress(Bd))
        assert r.c.header() == oracle.header(ref) and r.c.payload_bytes() == ref.payload_bytes()


def test_admission_limits_memory_and_slots(pool):
    """A tight arena and few slots force waiting; every result is still exact
    and no more than max_inflight requests were ever batched together."""
    import paper_1303_0270_amd as c
    from paper_1303_0270_amd import serve
    specs, mats = pool
    seed = W.seed_for(5, 4)
    reqs = serve.make_requests(mats, 120, None, seed, mm_frac=0.2)
    biggest = max(serve.request_footprint(r, mats) for r in reqs)
    srv = serve.Server(mats, arena_bytes=2 * biggest, streams=2, max_inflight=4, max_batch=4)
    stats = srv.run(reqs)
    srv.close()
    per_launch = {}
    for r in reqs:
        per_launch.setdefault(r.launch, []).append(r)
    assert max(len(v) for v in per_launch.values()) <= 4
    assert all(sum(r.footprint for r in v) <= 2 * biggest for v in per_launch.values())
    assert stats["launches"] >= 120 // 4
    check_alone(c, mats, reqs)


def test_oversized_request_is_rejected(pool):
    from paper_1303_0270_amd import serve
    specs, mats = pool
    reqs = serve.make_requests(mats, 5, None, W.seed_for(5, 5), mm_frac=0.0)
    srv = serve.Server(mats, arena_bytes=16, streams=1)
    with pytest.raises(ValueError):
        srv.run(reqs)
    srv.close()
