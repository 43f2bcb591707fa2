"""Measurements beside the main benchmark line: the dense compressed GEMM
(8192^3, A in [0, 2^6), B in [-2^3, 2^3)), the batched matvec and the serving
loop.  Called by bench.py after its timed steps."""
from __future__ import annotations

import time

import ccm_workloads as W

I8_PEAK_TOPS = 5000.0


def gemm(torch, ccm, n=8192, reps=3):
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
    ops = 2.0 * n * n * n
    return {"workload": f"{n}x{n}x{n}, A b={A.bits} unsigned, B b={B.bits} signed",
            "result_bits": C.bits, "result_signed": C.is_signed,
            "plan_ms": round(tp * 1e3, 3), "repack_ms": round(tk * 1e3, 3),
            "tops": round(ops / tp / 1e12, 2),
            "frac_i8_mfma": round(ops / tp / 1e12 / I8_PEAK_TOPS, 4)}


def run_extras(torch, ccm):
    out = {}
    t0 = time.perf_counter()
    out["gemm"] = gemm(torch, ccm)
    out["gemm"]["wall_s"] = round(time.perf_counter() - t0, 2)
    torch.cuda.empty_cache()
    return out
