"""Serving loop: every request's result in the mix equals the same request
run alone (bit for bit), sampled requests equal the oracle, and admission
holds requests back when slots or memory run out."""
import numpy as np
import pytest

import ccm_workloads as W
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "gpu tests need a GPU"


@pytest.fixture(scope="module")
def pool():
    from paper_1303_0270_amd import serve
    specs = W.serving_pool(48e6, max_elems=2e6)
    return specs, serve.make_pool(specs)


def check_alone(c, pool_mats, reqs):
    for r in reqs:
        a = pool_mats[r.mat]
        if r.kind == "mv":
            assert torch.equal(r.y, c.matvec(a, r.x)), r.rid
        else:
            alone = c.matmul(a, r.b)
            assert r.c.header() == alone.header() and \
                r.c.payload_bytes() == alone.payload_bytes(), r.rid


def check_oracle(specs, pool_mats, reqs, seed, count=8):
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
    srv = serve.Server(mats, arena_bytes=1 << 30, streams=3, max_inflight=64, max_batch=32)
    stats = srv.run(reqs)
    srv.close()
    assert stats["requests"] == 300 and all(np.isfinite(r.done) for r in reqs)
    assert stats["launches"] < 300 or qps  # burst arrivals are batched
    assert all(r.done >= r.arrival - 1e-4 for r in reqs)
    check_alone(c, mats, reqs)
    check_oracle(specs, mats, reqs, seed)


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
