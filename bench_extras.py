"""Measurements beside the main benchmark line: Method 2 (variable length
blocks) matvec on the paper's Beta bit-length distributions, the dense
compressed GEMM (8192^3, A in [0, 2^6), B in [-2^3, 2^3)), the batched matvec,
the serving loop and float matrices in fixed point.  Called by bench.py after
its timed steps."""
from __future__ import annotations

import time

import ccm_workloads as W

I8_PEAK_TOPS = 5000.0


def gemm(torch, ccm, n=8192, reps=3, i8_peak_measured=None):
    a_s, b_s = W.dense_gemm(n)
    A = ccm.generate(a_s.rows, a_s.cols, a_s.lo, a_s.hi, a_s.seed, a_s.stream)
    B = ccm.generate(b_s.rows, b_s.cols, b_s.lo, b_s.hi, b_s.seed, b_s.stream)
    scratch = torch.empty(ccm.matmul_scratch_bytes(A, B), dtype=torch.uint8, device="cuda")
    ccm.matmul(A, B, scratch)  # warm-up
    torch.cuda.synchronize()
    t_plan, t_pack = [], []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        C, scratch = ccm.matmul_plan(A, B, scratch)
        e[1].record()
        ccm.matmul_pack(A, B, C, scratch)
        e[2].record()
        torch.cuda.synchronize()
        t_plan.append(e[0].elapsed_time(e[1]) * 1e-3)
        t_pack.append(e[1].elapsed_time(e[2]) * 1e-3)
    tp, tk = min(t_plan), min(t_pack)
    # the whole product enqueued with no host wait (width decided on the device)
    ws = ccm.async_ws()
    payload = torch.empty(ccm.matmul_capacity(A, B), dtype=torch.uint8, device="cuda")
    ccm.matmul_async(A, B, scratch=scratch, ws=ws, payload=payload).get()
    t_async = []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        p = ccm.matmul_async(A, B, scratch=scratch, ws=ws, payload=payload)
        e[1].record()
        torch.cuda.synchronize()
        Ca = p.get()
        t_async.append(e[0].elapsed_time(e[1]) * 1e-3)
    assert Ca.header() == C.header()
    ta = min(t_async)
    ops = 2.0 * n * n * n
    out = {"workload": f"{n}x{n}x{n}, A b={A.bits} unsigned, B b={B.bits} signed",
           "result_bits": C.bits, "result_signed": C.is_signed,
           "plan_ms": round(tp * 1e3, 3), "repack_ms": round(tk * 1e3, 3),
           "async_total_ms": round(ta * 1e3, 3),
           "tops": round(ops / tp / 1e12, 2),
           "frac_i8_mfma": round(ops / tp / 1e12 / I8_PEAK_TOPS, 4)}
    if i8_peak_measured:
        out["frac_i8_mfma_measured_peak"] = round(ops / tp / 1e12 / i8_peak_measured, 4)
    out["library_int8_gemm"] = library_int8_gemm(torch, ccm, A, B, C, reps)
    return out


def library_int8_gemm(torch, ccm, A, B, C, reps):
    """Reference point: the vendor int8 GEMM (torch._int_mm, hipBLASLt) on the
    same operands already decoded to dense int8 (no decoding, no range, no
    packing), B stored K-contiguous like the B^T the MFMA path decodes.
    Checked against the packed result on the first 64 rows."""
    if not hasattr(torch, "_int_mm"):
        return None
    a8 = ccm.decompress(A).to(torch.int8)
    bt8 = ccm.decompress(B).to(torch.int8).t().contiguous()
    b8 = bt8.t()  # K x N view of N x K storage
    r = torch._int_mm(a8, b8)
    torch.cuda.synchronize()
    same = bool(torch.equal(r[:64].to(torch.int64), ccm.decompress(C)[:64]))
    ts = []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        r = torch._int_mm(a8, b8)
        e[1].record()
        torch.cuda.synchronize()
        ts.append(e[0].elapsed_time(e[1]) * 1e-3)
    t = min(ts)
    n = a8.shape[0]
    del a8, bt8, b8, r
    torch.cuda.empty_cache()
    return {"kernel": "torch._int_mm (hipBLASLt), dense int8 operands", "ms": round(t * 1e3, 3),
            "tops": round(2.0 * n * n * n / t / 1e12, 2), "first_64_rows_equal": same}


def batched(torch, ccm, reps=30):
    """4096 matrices (32..2048 x 32..2048, widths 1..24): one captured graph
    launch of the persistent batched kernel vs 4096 per-call launches."""
    import numpy as np
    items = W.batched()
    mats = [ccm.generate(it.a.rows, it.a.cols, it.a.lo, it.a.hi, it.a.seed, it.a.stream)
            for it in items]
    xs, ys = [], []
    for it in items:
        x = torch.empty(it.x.n, dtype=torch.int32, device="cuda")
        ccm.fill_uniform(x, it.x.lo, it.x.hi, it.x.seed, it.x.stream)
        xs.append(x)
        ys.append(torch.empty(it.a.rows, dtype=torch.int64, device="cuda"))
    batch = ccm.Batch(mats)
    batch.set_io(xs, ys)
    info = batch.info()
    for _ in range(3):
        batch.run(use_graph=True)
    torch.cuda.synchronize()
    lat = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        batch.run(use_graph=True)
        e1.record()
        torch.cuda.synchronize()
        lat.append(e0.elapsed_time(e1) * 1e-3)
    # the plain per-call path: one ccm_matvec launch per matrix, arguments
    # marshalled beforehand (the timed loop is the C calls and their launches)
    go = [ccm.matvec_launcher(m, x, y) for m, x, y in zip(mats, xs, ys)]
    for f in go[:64]:
        f()
    torch.cuda.synchronize()
    walls, gpus = [], []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record()
        for f in go:
            f()
        e1.record()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - w0)
        gpus.append(e0.elapsed_time(e1) * 1e-3)
    wall, per_call_gpu = min(walls), min(gpus)
    nbytes = info["packed_bytes"]
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
    out = {"workload": f"{len(items)} matrices, rows/cols 32..2048, widths 1..24, int32 x",
           "packed_bytes": nbytes, "items": info["items"],
           "graph_launch_p50_ms": round(p50 * 1e3, 3), "graph_launch_p99_ms": round(p99 * 1e3, 3),
           "graph_gbs": round(nbytes / p50 / 1e9, 1),
           "graph_frac_hbm": round(nbytes / p50 / 1e9 / 8000.0, 4),
           "per_call_wall_ms": round(wall * 1e3, 3), "per_call_gpu_ms": round(per_call_gpu * 1e3, 3),
           "per_call_us_per_launch": round(per_call_gpu / len(go) * 1e6, 2),
           "per_call_gbs": round(nbytes / per_call_gpu / 1e9, 1),
           "per_call_note": "4096 ccm_matvec calls with pre-marshalled arguments, back to back "
                            "on one stream; gpu = events around them",
           "speedup_vs_per_call": round(per_call_gpu / p50, 2)}
    batch.close()
    return out


def serving(torch, ccm, target_bytes=200e9, count=2000, log=None):
    """Resident pool (~200 GB packed, 1e4..1e9 elements, widths 1..20),
    requests 90% matvec / 10% small matmul: saturation throughput from a
    burst, then Poisson arrivals at 50/80/95% of it."""
    from paper_1303_0270_amd import serve
    specs = W.serving_pool(target_bytes)
    t0 = time.perf_counter()
    pool = serve.make_pool(specs)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    packed = sum(64 + 8 * m.words for m in pool)
    as_int32 = sum(4 * m.rows * m.cols for m in pool)
    if log:
        log(f"pool: {len(pool)} matrices, {packed / 1e9:.1f} GB packed, generated in {gen_s:.1f} s")
    free, total = torch.cuda.mem_get_info()
    arena = max(1 << 30, free - (16 << 30))
    srv = serve.Server(pool, arena_bytes=arena, streams=4, max_inflight=512, max_batch=256)
    seed = W.seed_for(5, 2)
    # warm-up, untimed: one matvec per pool matrix (loads every kernel the
    # pool's shapes and widths use, as a server does at start), then a short
    # burst through the serving loop
    xw = torch.ones(max(m.cols for m in pool), dtype=torch.int32, device="cuda")
    yw = torch.empty(max(m.rows for m in pool), dtype=torch.int64, device="cuda")
    for m in pool:
        ccm.matvec(m, xw[: m.cols], yw[: m.rows])
    torch.cuda.synchronize()
    del xw, yw
    warm = serve.make_requests(pool, 200, None, seed, first_rid=10_000_000)
    srv.run(warm)
    burst = serve.make_requests(pool, count, None, seed)
    sat = srv.run(burst)
    del burst
    out = {"pool_matrices": len(pool), "pool_packed_gb": round(packed / 1e9, 2),
           "pool_as_int32_gb": round(as_int32 / 1e9, 2), "arena_gb": round(arena / 1e9, 1),
           "saturation": sat, "load": {}}
    for frac in (0.5, 0.8, 0.95):
        qps = frac * sat["throughput_rps"]
        reqs = serve.make_requests(pool, count, qps, seed + int(frac * 100),
                                   first_rid=int(frac * 1_000_000))
        st = srv.run(reqs)
        st["offered_qps"] = round(qps, 1)
        out["load"][f"{int(frac * 100)}%"] = st
        if log:
            log(f"serving at {frac:.0%}: p50 {st['p50_ms']} ms p99 {st['p99_ms']} ms")
        del reqs
    srv.close()
    del pool
    torch.cuda.empty_cache()
    return out


# VALU instructions per element of the staged VLB walk when the pair fits 32
# bits (funnel shift, length mask, extract, multiply-add, two position adds,
# word index, window compare and select, width test, LDS address).
VLB_VALU_PER_ELEM = 11
VALU_LANE_OPS = 256 * 64 * 2.4e9  # lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz


def vlb(torch, ccm, reps=20):
    """Method 2 matvec on 16384 x 16384 matrices whose bit-lengths follow the
    paper's Beta distributions (two compressed copies used in turn, so the
    256 MB last-level cache holds neither), with the Method 1 width of the
    same matrix and both efficiencies (Eq. 15, Eq. 17)."""
    import numpy as np
    out = {}
    for name in W.VLB_BETAS:
        spec, xs = W.vlb_sweep(name)
        A = spec.dense_device(ccm.fill_uniform, torch)
        n = spec.rows * spec.cols
        ccm.method_info(A)  # warm-up
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        info = ccm.method_info(A)  # blocking: one pass plus the readback
        t_sel = time.perf_counter() - c0
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        g0 = ccm.vlb_compress(A)
        ev[1].record()
        torch.cuda.synchronize()
        t_comp = ev[0].elapsed_time(ev[1]) * 1e-3
        g1 = ccm.vlb_compress(A)
        sm_bits, _ = ccm.width(int(g0.vmin), int(g0.vmax))
        del A
        x = torch.from_numpy(xs.dense()).to(torch.int32).cuda()
        y = torch.empty(spec.rows, dtype=torch.int64, device="cuda")
        go = [ccm.vlb_matvec_launcher(g, x, y) for g in (g0, g1)]
        for i in range(4):
            go[i % 2]()
        torch.cuda.synchronize()
        ts = []
        for i in range(reps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record()
            go[i % 2]()
            e[1].record()
            torch.cuda.synchronize()
            ts.append(e[0].elapsed_time(e[1]) * 1e-3)
        t = float(np.median(ts))
        stream = 8 * g0.words
        alu_t = n * VLB_VALU_PER_ELEM / VALU_LANE_OPS
        out[name] = {
            "workload": f"{spec.rows}x{spec.cols}, bit-lengths Beta({spec.a1:g}, {spec.b1:g}) on [1, 64]",
            "k": g0.k, "avg_bits_per_elem": round(g0.nbits / n, 3), "gmax_bits": g0.gmax,
            "eta2_vlb": round(1 - g0.nbits / (64 * n), 4), "eta1_sm": round(1 - sm_bits / 64, 4),
            "method_chosen": info["method"],
            "select_ms": round(t_sel * 1e3, 3),
            "select_gb_s_dense": round(8 * n / t_sel / 1e9, 1),
            "index_bytes": g0.index_bytes, "stream_bytes": stream,
            "compress_ms": round(t_comp * 1e3, 2),
            "matvec_us": round(t * 1e6, 1),
            "matvec_gb_s": round(stream / t / 1e9, 1),
            "matvec_gb_s_with_index": round((stream + g0.index_bytes) / t / 1e9, 1),
            "gelem_s": round(n / t / 1e9, 1),
            "frac_hbm": round(stream / t / 8e12, 4),
            "frac_alu_model": round(alu_t / t, 4),
        }
        del g0, g1, go
        torch.cuda.empty_cache()
    return out


def transposed(torch, ccm, reps=10):
    """y = A^T x (the column-major matrix's y = A x) on the 16384 x 16384
    unsigned sweep matrices, beside y = A x on the same payload; enough copies
    that each call streams from HBM (their total > 512 MB), launched back to
    back with pre-marshalled arguments."""
    import numpy as np
    out = {}
    for k in W.SWEEP_WIDTHS:
        a_s, _, x_s, _ = W.sweep(k, False)
        one = 8 * ccm.words(a_s.rows, a_s.cols, k)
        ncopy = max(2, -(-(512 << 20) // one))
        mats = [ccm.generate(a_s.rows, a_s.cols, a_s.lo, a_s.hi, a_s.seed, a_s.stream)
                for _ in range(ncopy)]
        x = torch.empty(a_s.rows, dtype=torch.int32, device="cuda")
        ccm.fill_uniform(x, x_s.lo, x_s.hi, x_s.seed, x_s.stream)
        y = torch.empty(a_s.cols, dtype=torch.int64, device="cuda")
        res = {}
        for name, tr in (("matvec_t", True), ("matvec", False)):
            # arguments marshalled once: back-to-back launches, per-call time
            # = events around one pass over the copies / copies
            go = [ccm.matvec_launcher(m, x, y, transposed=tr) for m in mats]
            for i in range(2 * ncopy):
                go[i % ncopy]()
            torch.cuda.synchronize()
            ts = []
            for i in range(reps):
                e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                e[0].record()
                for f in go:
                    f()
                e[1].record()
                torch.cuda.synchronize()
                ts.append(e[0].elapsed_time(e[1]) * 1e-3 / ncopy)
            t = float(np.median(ts))
            res[name] = {"us": round(t * 1e6, 1), "gb_s": round(one / t / 1e9, 1)}
        res["packed_mb"] = round(one / 1e6, 1)
        out[f"k{k}"] = res
        del mats
        torch.cuda.empty_cache()
    return out


def floats(torch, ccm, n=16384, reps=10):
    """Floats in fixed point (Conclusion): a 16384 x 16384 float32 matrix
    (v = m 2^e, m in [-2^23, 2^23), e in [-20, 0]) kept to p = 8, 12 and 16
    significant bits of its largest magnitude: compression (largest
    magnitude, quantization with the exact range, packing), size against
    float32, the largest rounding error, y = V x with x kept to 14
    significant bits (the int32 fast matvec path) per call and the packed
    matvec kernels alone, beside a dense float32 matvec (torch.mv)."""
    import numpy as np
    ms, es, xs = W.float_matrix(n)
    mt = torch.empty((n, n), dtype=torch.int32, device="cuda")
    et = torch.empty((n, n), dtype=torch.int32, device="cuda")
    ccm.fill_uniform(mt, ms.lo, ms.hi, ms.seed, ms.stream)
    ccm.fill_uniform(et, es.lo, es.hi, es.seed, es.stream)
    V = torch.ldexp(mt.to(torch.float32), et.to(torch.float32))
    del mt, et
    xm = torch.empty(n, dtype=torch.int32, device="cuda")
    ccm.fill_uniform(xm, xs.lo, xs.hi, xs.seed, xs.stream)
    x = torch.ldexp(xm.to(torch.float32), torch.full_like(xm, -23, dtype=torch.float32))
    torch.cuda.synchronize()
    out = {"workload": f"{n}x{n} float32, v = m 2^e, m uniform in [-2^23, 2^23), e in [-20, 0];"
                       " x in [-1, 1)", "float32_bytes": 4 * n * n}

    def timed(fn, k=reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(k):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    for p in (8, 12, 16):
        t_c = timed(lambda: ccm.compress_float(V, sig_bits=p), 3)
        m = ccm.compress_float(V, sig_bits=p)
        back = ccm.decompress_float(m, torch.float32)
        err = float((back.double() - V.double()).abs().max())
        del back
        t_mv = timed(lambda: ccm.matvec_float(m, x, x_sig_bits=14))
        # the packed matvec alone: the quantized x, launches back to back
        xq, _, _ = ccm.quantize(x, ccm.float_frac_bits(ccm.float_absmax(x), 14),
                                dtype=torch.int32)
        y = torch.empty(n, dtype=torch.int64, device="cuda")
        go = ccm.matvec_launcher(m, xq, y)
        t_k = timed(lambda: [go() for _ in range(10)]) / 10
        pb = 8 * m.words
        out[f"p{p}"] = {"frac_bits": m.frac_bits, "bits": m.bits, "packed_bytes": pb,
                        "vs_float32": round(pb / (4 * n * n), 4),
                        "max_abs_error": err, "error_bound": 2.0 ** (-m.frac_bits - 1),
                        "compress_ms": round(t_c * 1e3, 3),
                        "compress_gb_s_float32_in": round(4 * n * n / t_c / 1e9, 1),
                        "matvec_float_call_us": round(t_mv * 1e6, 1),
                        "matvec_kernels_us": round(t_k * 1e6, 1),
                        "matvec_gb_s_packed": round(pb / t_k / 1e9, 1)}
        del m
        torch.cuda.empty_cache()
    yd = torch.empty(n, dtype=torch.float32, device="cuda")
    t_d = timed(lambda: [torch.mv(V, x, out=yd) for _ in range(10)]) / 10
    out["dense_float32_mv"] = {"us": round(t_d * 1e6, 1), "gb_s": round(4 * n * n / t_d / 1e9, 1),
                               "kernel": "torch.mv (rocBLAS gemv), float32"}
    return out


def run_extras(torch, ccm, log=None, i8_peak_measured=None):
    out = {}
    t0 = time.perf_counter()
    out["transposed"] = transposed(torch, ccm)
    out["transposed"]["wall_s"] = round(time.perf_counter() - t0, 2)
    if log:
        log("transposed done")
    t0 = time.perf_counter()
    out["vlb"] = vlb(torch, ccm)
    out["vlb"]["wall_s"] = round(time.perf_counter() - t0, 2)
    torch.cuda.empty_cache()
    if log:
        log("vlb done")
    t0 = time.perf_counter()
    out["gemm"] = gemm(torch, ccm, i8_peak_measured=i8_peak_measured)
    out["gemm"]["wall_s"] = round(time.perf_counter() - t0, 2)
    torch.cuda.empty_cache()
    if log:
        log("gemm done")
    t0 = time.perf_counter()
    out["batched"] = batched(torch, ccm)
    out["batched"]["wall_s"] = round(time.perf_counter() - t0, 2)
    torch.cuda.empty_cache()
    if log:
        log("batched done")
    t0 = time.perf_counter()
    out["floats"] = floats(torch, ccm)
    out["floats"]["wall_s"] = round(time.perf_counter() - t0, 2)
    torch.cuda.empty_cache()
    if log:
        log("floats done")
    t0 = time.perf_counter()
    out["serving"] = serving(torch, ccm, log=log)
    out["serving"]["wall_s"] = round(time.perf_counter() - t0, 2)
    if log:
        log("serving done")
    return out
