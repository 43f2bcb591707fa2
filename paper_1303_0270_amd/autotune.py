"""Autotuner for the batched matvec: per field width, picks the rows per work
item ("tile_rows") and the rows each lane keeps in flight (1, 2 or 4) that give
the fastest graph launch on a synthetic batch of that width, and writes the
table read by ccm_batch_create.

usage: python -m paper_1303_0270_amd.autotune [--out PATH] [--widths 1-24]
       [--count 128] [--reps 7]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import tempfile

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune", "gfx950.json")
TILE_ROWS = (64, 128, 256, 512, 1024)


def parse_widths(text: str):
    out = []
    for part in text.split(","):
        if "-" in part:
            a, b = part.split("-")
            out.extend(range(int(a), int(b) + 1))
        else:
            out.append(int(part))
    return out


def time_batch(torch, ccm, mats, xs, ys, table_path, reps):
    batch = ccm.Batch(mats, tune_json=table_path)
    batch.set_io(xs, ys)
    batch.run(use_graph=True)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        batch.run(use_graph=True)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    batch.close()
    return statistics.median(ts)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--widths", default="1-24")
    ap.add_argument("--count", type=int, default=128)
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import ccm_workloads as W
    import paper_1303_0270_amd as ccm

    seed = W.seed_for(4, 7)
    table = {"device": torch.cuda.get_device_name(0), "widths": {}}
    tmpdir = tempfile.mkdtemp()
    for b in parse_widths(args.widths):
        rows = W.uniform(seed, 2 * b, 0, args.count, 32, 2049)
        cols = W.uniform(seed, 2 * b + 1, 0, args.count, 32, 2049)
        mats, xs, ys = [], [], []
        for t in range(args.count):
            mats.append(ccm.generate(int(rows[t]), int(cols[t]), 0, 1 << b, seed, 1000 * b + t))
            x = torch.empty(int(cols[t]), dtype=torch.int32, device="cuda")
            ccm.fill_uniform(x, -(1 << 15), 1 << 15, seed, 500000 + 1000 * b + t)
            xs.append(x)
            ys.append(torch.empty(int(rows[t]), dtype=torch.int64, device="cuda"))
        nbytes = sum(8 * m.words for m in mats)
        best = None
        for tile in TILE_ROWS:
            for rif in ((1, 2, 4) if b <= 8 else (1, 2) if b <= 16 else (1,)):
                path = os.path.join(tmpdir, f"t{b}_{tile}_{rif}.json")
                with open(path, "w") as f:
                    json.dump({"widths": {str(b): {"tile_rows": tile, "rows_in_flight": rif}}}, f)
                t = time_batch(torch, ccm, mats, xs, ys, path, args.reps)
                if best is None or t < best[0]:
                    best = (t, tile, rif)
        table["widths"][str(b)] = {"tile_rows": best[1], "rows_in_flight": best[2],
                                   "us": round(best[0] * 1e6, 1),
                                   "gbs": round(nbytes / best[0] / 1e9, 1)}
        print(f"b={b:2d} tile_rows={best[1]:5d} rows_in_flight={best[2]} "
              f"{best[0] * 1e6:8.1f} us {nbytes / best[0] / 1e9:7.1f} GB/s", flush=True)
        del mats, xs, ys
        torch.cuda.empty_cache()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
