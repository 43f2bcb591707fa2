"""Benchmark of the compressed-matrix hot path on one MI355X.

Workload: the bandwidth sweep -- 16384 x 16384 matrices uniform in [0, 2^k)
and in [-2^(k-1), 2^(k-1)) for k in {1, 3, 7, 12, 17, 31} (twelve matrices),
a second matrix of each kind for add, and an int32 x uniform in
[-2^15, 2^15).  All inputs are seeded synthetic data generated on the device
(SplitMix64) and resident in HBM before the timed region.

One step runs every operation of the path over the twelve matrices, in
phases: width + compress (from the dense int64 input), matvec, add (one
pass: pack at the headers' bound width with the exact range folded in; the
asynchronous form, its width decided on the device and the twelve headers
read back once all adds are enqueued), scale by 7, decompress and 1000
element gets.  The reported
value is the packed-matvec bandwidth: the packed bytes of A (8*W per matrix)
over the time of the matvec phase, taken with a pair of HIP events on the
launch stream around the twelve back-to-back launches (even steps); odd steps
put one event between neighbouring launches for the per-width breakdown, and
each such marker adds a few microseconds to its interval.  Each phase touches
gigabytes before a matrix is read again, so the 256 MB last-level cache does
not hold A between its compression and its matvec.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-extras] [--profile] [--extras-only NAMES]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)
METRIC = ("packed-matvec HBM GB/s (% peak) + Gelem/s vs dense int32; "
          "batched p50/p99 latency")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: compress and matvec sweep, comparisons")
    ap.add_argument("--matvec-only", action="store_true",
                    help="counter runs: the twelve packed matrices generated directly on the "
                         "device, K matvec sweeps, then a 1 GiB calibration copy")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="write the HBM-traffic summary of two rocprofv3 --pmc runs of "
                         "--matvec-only (DIR/fetch, DIR/write) to --counters-out; no GPU use")
    ap.add_argument("--counters-out", default=os.path.join("profiles",
                                                           "matvec_sweep_hbm_counters.md"))
    ap.add_argument("--summarize-trace", metavar="CSV",
                    help="write the kernel-time summary of a rocprofv3 --kernel-trace --stats "
                         "run of this benchmark (its kernel_stats.csv) to --trace-out; no GPU use")
    ap.add_argument("--trace-json", metavar="FILE",
                    help="the JSON line the profiled run printed (matvec event times, compared)")
    ap.add_argument("--trace-cmd", default="", help="the profiled command, recorded in the summary")
    ap.add_argument("--trace-out", default=os.path.join("profiles", "sweep_step_kernels.md"))
    ap.add_argument("--trace-title", default="", help="summary title (default: the step's)")
    ap.add_argument("--trace-note", default="", help="summary description (default: the step's)")
    ap.add_argument("--summarize-traffic", metavar="DIR",
                    help="write the HBM traffic per kernel of two rocprofv3 --pmc runs (DIR/fetch "
                         "FETCH_SIZE, DIR/write WRITE_SIZE) of any command that ends with a "
                         "1 GiB device copy, for kernels matching --traffic-kernels; no GPU use")
    ap.add_argument("--traffic-kernels", default=".", help="regex of kernel names to list")
    ap.add_argument("--traffic-out", default=os.path.join("profiles", "traffic.md"))
    ap.add_argument("--traffic-title", default="HBM traffic per kernel")
    ap.add_argument("--traffic-cmd", default="", help="the profiled command, recorded")
    ap.add_argument("--traffic-note", default="")
    ap.add_argument("--extras-only", metavar="NAMES",
                    help="run only these measurements of bench_extras (comma list of "
                         "transposed, vlb, gemm, batched, serving) and print their JSON; for "
                         "profiling the kernels they launch")
    return ap.parse_args()


# Sources whose change makes recorded hardware counters of the matvec kernels stale.
MATVEC_SOURCES = ["paper_1303_0270_amd/csrc/matvec_impl.hpp", "paper_1303_0270_amd/csrc/matvec.hip",
                  "paper_1303_0270_amd/csrc/matvec_w1.hip", "paper_1303_0270_amd/csrc/matvec_w2.hip",
                  "paper_1303_0270_amd/csrc/matvec_w3.hip", "paper_1303_0270_amd/csrc/matvec_w4.hip",
                  "paper_1303_0270_amd/csrc/ccm_internal.hpp",
                  "paper_1303_0270_amd/csrc/group_codec.hpp", "paper_1303_0270_amd/build.py"]
COUNTERS_MD = os.path.join(ROOT, "profiles", "matvec_sweep_hbm_counters.md")
# FETCH_SIZE / WRITE_SIZE (KiB) per byte moved, from a plain 1 GiB device copy in the same run
# (reads 2^30 bytes, writes 2^30 bytes): the factors turn the counters into bytes.


def matvec_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in MATVEC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per matvec launch of the sweep, from the committed counter
    summary; None when there is none or the matvec sources changed since."""
    import re
    if not os.path.exists(COUNTERS_MD):
        return None
    text = open(COUNTERS_MD).read()
    m = re.search(r"matvec source hash: `([0-9a-f]+)`", text)
    t = re.search(r"HBM bytes per launch \(mean over the sweep\): ([0-9.]+)", text)
    if not m or not t or m.group(1) != matvec_source_hash():
        return None
    return float(t.group(1))


def summarize_counters(src_dir, out_path):
    """Builds the counter summary from rocprofv3 --pmc FETCH_SIZE and
    WRITE_SIZE runs of `bench.py --matvec-only` (CSV output under
    src_dir/fetch and src_dir/write)."""
    import csv
    import glob

    def per_kernel(sub, counter):
        vals = {}
        for f in glob.glob(os.path.join(src_dir, sub, "**", "*counter_collection.csv"),
                           recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals

    fetch = per_kernel("fetch", "FETCH_SIZE")
    write = per_kernel("write", "WRITE_SIZE")
    copy_f = [v for k, vs in fetch.items() if "copyBuffer" in k for v in vs]
    copy_w = [v for k, vs in write.items() if "copyBuffer" in k for v in vs]
    gib_kib = float(1 << 20)
    ff = gib_kib / max(copy_f) if copy_f else None  # bytes read per FETCH_SIZE KiB / 1024
    fw = gib_kib / max(copy_w) if copy_w else None
    rows = []
    for name in sorted(fetch):
        if "k_matvec" not in name:
            continue
        f_kib = sum(fetch[name]) / len(fetch[name])
        w_kib = sum(write.get(name, [0.0])) / max(1, len(write.get(name, [])))
        rows.append((name.split("(")[0].replace("void ", ""), len(fetch[name]), f_kib, w_kib,
                     1024 * (f_kib * ff + w_kib * fw)))
    mean = sum(r[4] for r in rows) / len(rows)
    lines = [
        "# HBM traffic of the matvec kernels: 16384 x 16384 bandwidth sweep",
        "",
        "Commands (repo root on the MI355X box; rocprofv3 run from /tmp with TMPDIR=/tmp):",
        "",
        f"    timeout -s KILL 60 rocprofv3 --pmc FETCH_SIZE -d {src_dir}/fetch -o fetch \\",
        "        --output-format csv -- python3 bench.py --matvec-only --steps 1 --warmup 0",
        f"    timeout -s KILL 60 rocprofv3 --pmc WRITE_SIZE -d {src_dir}/write -o write \\",
        "        --output-format csv -- python3 bench.py --matvec-only --steps 1 --warmup 0",
        f"    python3 bench.py --summarize-counters {src_dir}",
        "",
        "`--matvec-only` generates the twelve packed sweep matrices (k in {1,3,7,12,17,31}, "
        "unsigned and signed) on the device, runs one matvec per matrix, then a plain 1 GiB "
        "device copy used to calibrate the counters.",
        "",
        f"Calibration: the 1 GiB copy reads FETCH_SIZE {max(copy_f):.0f} KiB and writes WRITE_SIZE "
        f"{max(copy_w):.0f} KiB; bytes = KiB x 1024 x {ff:.3f} (fetch) and x {fw:.3f} (write).",
        "",
        f"matvec source hash: `{matvec_source_hash()}` (sha256 prefix of the matvec sources; "
        "bench.py reports `roofline.traffic` only while it matches)",
        "",
        "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (calibrated) |",
        "|---|---|---|---|---|",
    ]
    for r in rows:
        lines.append(f"| `{r[0]}` | {r[1]} | {r[2]:.0f} | {r[3]:.0f} | {r[4]:.0f} |")
    lines += ["", f"HBM bytes per launch (mean over the sweep): {mean:.0f}", ""]
    with open(out_path, "w") as f:
        f.write("\n".join(lines))
    print(out_path)


def summarize_traffic(src_dir, out_path, pattern, title, cmd, note):
    """HBM bytes per dispatch of the kernels matching `pattern`, from
    rocprofv3 --pmc FETCH_SIZE (src_dir/fetch) and WRITE_SIZE (src_dir/write)
    runs of one command, calibrated by that run's plain 1 GiB device copy."""
    import csv
    import glob
    import re

    def per_kernel(sub, counter):
        vals = {}
        for f in glob.glob(os.path.join(src_dir, sub, "**", "*counter_collection.csv"),
                           recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals

    def short(name):
        return name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]

    fetch = per_kernel("fetch", "FETCH_SIZE")
    write = per_kernel("write", "WRITE_SIZE")
    copy_f = [v for k, vs in fetch.items() if "copyBuffer" in k for v in vs]
    copy_w = [v for k, vs in write.items() if "copyBuffer" in k for v in vs]
    gib_kib = float(1 << 20)
    ff, fw = gib_kib / max(copy_f), gib_kib / max(copy_w)
    rx = re.compile(pattern)
    lines = ["# " + title, "",
             "Commands (repo root on the MI355X box; rocprofv3 run from /tmp with TMPDIR=/tmp):",
             "", "    " + cmd.replace("\n", "\n    "), "", note, "",
             f"Calibration: the run's 1 GiB device copy reads FETCH_SIZE {max(copy_f):.0f} KiB and "
             f"writes WRITE_SIZE {max(copy_w):.0f} KiB; bytes = KiB x 1024 x {ff:.3f} (fetch) and "
             f"x {fw:.3f} (write).", "",
             "| kernel | dispatches | mean FETCH_SIZE KiB | mean WRITE_SIZE KiB | mean HBM bytes "
             "per dispatch (calibrated) | total HBM bytes |", "|---|---|---|---|---|---|"]
    for name in sorted(set(fetch) | set(write)):
        if not rx.search(name) or "copyBuffer" in name:
            continue
        fv, wv = fetch.get(name, [0.0]), write.get(name, [0.0])
        f_kib, w_kib = sum(fv) / len(fv), sum(wv) / len(wv)
        per = 1024 * (f_kib * ff + w_kib * fw)
        tot = 1024 * (sum(fv) * ff + sum(wv) * fw)
        lines.append(f"| `{short(name)}` | {max(len(fv), len(wv))} | {f_kib:.0f} | {w_kib:.0f} | "
                     f"{per:.0f} | {tot:.0f} |")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out_path)


def summarize_trace(stats_csv, out_path, bench_json=None, cmd="", title="", note=""):
    """Kernel-time table of a rocprofv3 --kernel-trace --stats run of this
    benchmark; with the run's JSON line, the matvec kernels' trace averages
    next to the HIP-event times bench.py measured in the same run."""
    import csv
    import re

    def short(name):
        if "FillFunctor" in name:
            return "torch fill_"
        return name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]

    rows = list(csv.DictReader(open(stats_csv)))
    title = title or "Kernel times: one benchmark step over the 16384 x 16384 bandwidth sweep"
    note = note or ("A step runs width + compress, matvec, add (asynchronous, one pass, the exact range "
                    "folded into the pack), scale by 7, "
                    "decompress and 1000 gets over the twelve sweep matrices (k in "
                    "{1,3,7,12,17,31}, unsigned and signed); the dense int32 comparison, the read "
                    "probe and a 1 GiB copy follow.")
    lines = ["# " + title, "",
             "Command (repo root on the MI355X box; rocprofv3 run from /tmp with TMPDIR=/tmp):", "",
             "    " + cmd, "", note, "",
             "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    if bench_json:
        d = json.loads(open(bench_json).read().strip().splitlines()[-1])
        lines += ["", "Matvec kernels: rocprofv3 average against the HIP-event time bench.py took "
                  "in the same run (`per_width[].matvec_us`).", "",
                  "| width | signed | trace avg us | bench event us |", "|---|---|---|---|"]
        for pw in d["per_width"]:
            sg = "true" if pw["signed"] else "false"
            pat = re.compile(r"k_matvec\w*<%d, %s" % (pw["bits"], sg))
            tr = [float(r["AverageNs"]) / 1e3 for r in rows if pat.search(r["Name"])]
            lines.append(f"| {pw['bits']} | {sg} | {tr[0]:.1f} | {pw['matvec_us']:.1f} |" if tr
                         else f"| {pw['bits']} | {sg} | - | {pw['matvec_us']:.1f} |")
        mv = [float(r["AverageNs"]) / 1e3 for r in rows if "k_matvec" in r["Name"]]
        lines += ["", "Per-width event intervals each include one event marker; the value "
                  "uses the even steps' pair of events around all twelve launches instead:", "",
                  f"* sum of the matvec kernels' trace averages: {sum(mv):.1f} us per sweep",
                  f"* bench matvec phase (event pair): {d['ops']['matvec']['ms_per_sweep'] * 1e3:.1f}"
                  f" us per sweep",
                  f"* bench value: {d['value']} GB/s (roofline frac {d['roofline']['frac']})"]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out_path)


class Timer:
    """HIP events on the current stream, accumulated per label."""

    def __init__(self, torch):
        self.torch = torch
        self.pending = []

    def span(self, label):
        torch = self.torch
        timer = self

        class _S:
            def __enter__(self_):
                self_.a = torch.cuda.Event(enable_timing=True)
                self_.b = torch.cuda.Event(enable_timing=True)
                self_.a.record()

            def __exit__(self_, *exc):
                self_.b.record()
                timer.pending.append((label, self_.a, self_.b))
        return _S()

    def chain(self, labels_and_calls):
        """Launches back to back with one event between neighbours: launch i
        is timed from the event before it to the event after it.  The events
        are created and the launches marshalled before the first record, so
        the host enqueues faster than the kernels run and no host gap lands
        inside an interval."""
        torch = self.torch
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(labels_and_calls) + 1)]
        evs[0].record()
        for i, (label, call) in enumerate(labels_and_calls):
            call()
            evs[i + 1].record()
            self.pending.append((label, evs[i], evs[i + 1]))

    def phase(self, label, calls):
        """Launches back to back between one pair of events (no marker between
        the kernels)."""
        torch = self.torch
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for call in calls:
            call()
        b.record()
        self.pending.append((label, a, b))

    def collect(self):
        out = {}
        for label, a, b in self.pending:
            out.setdefault(label, []).append(a.elapsed_time(b) * 1e-3)
        self.pending = []
        return out


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.counters_out)
        return
    if args.summarize_traffic:
        summarize_traffic(args.summarize_traffic, args.traffic_out, args.traffic_kernels,
                          args.traffic_title, args.traffic_cmd, args.traffic_note)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.trace_out, args.trace_json, args.trace_cmd,
                        args.trace_title, args.trace_note)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import ccm_workloads as W
    import paper_1303_0270_amd as ccm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.matvec_only:
        matvec_only(args, torch, W, ccm)
        return
    if args.extras_only:
        import bench_extras as X
        fns = {"transposed": X.transposed, "vlb": X.vlb, "gemm": X.gemm, "batched": X.batched,
               "serving": X.serving, "floats": X.floats}
        res = {}
        for name in args.extras_only.split(","):
            res[name] = fns[name](torch, ccm)
            torch.cuda.empty_cache()
            log(f"{name} done")
        # a plain 1 GiB device copy: calibrates FETCH_SIZE / WRITE_SIZE counter runs
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"extras_only": res}), flush=True)
        return
    bench_lib = ctypes.CDLL(os.path.join(ROOT, "paper_1303_0270_amd", "libccm_bench.so"))
    bench_lib.ccmb_dense_matvec_i32.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p]
    bench_lib.ccmb_read_bytes.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.c_int, ctypes.c_void_p]
    bench_lib.ccmb_mfma_i8_peak.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_void_p]
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    n = args.n

    # ---- resident inputs -------------------------------------------------
    cases = []
    x_spec = None
    for k in W.SWEEP_WIDTHS:
        for signed in (False, True):
            a_s, b_s, x_s, s = W.sweep(k, signed, n)
            x_spec = x_s
            dense = torch.empty((n, n), dtype=torch.int64, device="cuda")
            ccm.fill_uniform(dense, a_s.lo, a_s.hi, a_s.seed, a_s.stream)
            bden = torch.empty((n, n), dtype=torch.int64, device="cuda")
            ccm.fill_uniform(bden, b_s.lo, b_s.hi, b_s.seed, b_s.stream)
            bpk = ccm.compress(bden)
            del bden
            # the asynchronous add's workspace and pinned header buffer, reused
            # by every step (each step reads its results back before the next)
            cases.append({"k": k, "signed": signed, "spec": a_s, "dense": dense, "B": bpk,
                          "scale": s, "ws": ccm.async_ws(),
                          "host": torch.empty(64, dtype=torch.uint8, pin_memory=True)})
    x = torch.empty(n, dtype=torch.int32, device="cuda")
    ccm.fill_uniform(x, x_spec.lo, x_spec.hi, x_spec.seed, x_spec.stream)
    y = torch.empty(n, dtype=torch.int64, device="cuda")
    dec = torch.empty((n, n), dtype=torch.int64, device="cuda")
    rng = np.random.default_rng(W.seed_for(2, 3))
    gi = torch.from_numpy(rng.integers(0, n, 1000)).cuda()
    gj = torch.from_numpy(rng.integers(0, n, 1000)).cuda()
    torch.cuda.synchronize()
    log("inputs resident")

    timer = Timer(torch)

    nstep = [0]

    def step(profile=False):
        packed = []
        for c in cases:
            with timer.span(f"compress:{c['k']}:{int(c['signed'])}"):
                a = ccm.compress(c["dense"])
            packed.append(a)
        # Even steps time the twelve back-to-back launches as one phase (the
        # value); odd steps put one event between neighbouring launches for the
        # per-width breakdown -- each marker adds a few us to its interval.
        launches = [(f"matvec:{c['k']}:{int(c['signed'])}", ccm.matvec_launcher(a, x, y, stream))
                    for c, a in zip(cases, packed)]
        if nstep[0] % 2 == 0:
            timer.phase("matvec_phase", [go for _, go in launches])
        else:
            timer.chain(launches)
        nstep[0] += 1
        if profile:
            return packed
        # add with the result's width decided on the device (no host wait per
        # add, as the serving path runs it); the twelve results' headers are
        # read back once all are enqueued
        pend = []
        for c, a in zip(cases, packed):
            with timer.span(f"add:{c['k']}:{int(c['signed'])}"):
                pend.append(ccm.add_async(a, c["B"], ws=c["ws"], host=c["host"]))
        for c, p in zip(cases, pend):
            c["sum"] = p.get()
        for c, a in zip(cases, packed):
            with timer.span(f"scale:{c['k']}:{int(c['signed'])}"):
                c["scaled"] = ccm.scale(a, c["scale"])
        for c, a in zip(cases, packed):
            with timer.span(f"decompress:{c['k']}:{int(c['signed'])}"):
                ccm.decompress(a, out=dec)
            with timer.span(f"get:{c['k']}:{int(c['signed'])}"):
                ccm.gather(a, gi, gj, sync=False)
        return packed

    for _ in range(args.warmup):
        step(args.profile)
    torch.cuda.synchronize()
    timer.collect()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        packed = step(args.profile)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = timer.collect()
    log(f"{args.steps} timed steps: {wall / args.steps * 1e3:.1f} ms/step")

    # ---- matvec roofline -------------------------------------------------
    per_width = []
    sweep_bytes = 0.0
    for c, a in zip(cases, packed):
        ts = times.get(f"matvec:{c['k']}:{int(c['signed'])}", [float("nan")])
        t = float(np.mean(ts))
        nbytes = 8 * a.words
        sweep_bytes += nbytes
        per_width.append({"k": c["k"], "signed": c["signed"], "bits": a.bits,
                          "packed_bytes": nbytes, "matvec_us": round(t * 1e6, 2),
                          "gbs": round(nbytes / t / 1e9, 1),
                          "frac_hbm": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4),
                          "gelem_s": round(n * n / t / 1e9, 1)})
    phases = times.get("matvec_phase")
    if not phases:  # a single timed step: sum its per-launch intervals
        phases = [sum(float(np.sum(times[f"matvec:{c['k']}:{int(c['signed'])}"]))
                      for c in cases)]
    tot_t = float(np.sum(phases))
    value = sweep_bytes * len(phases) / tot_t / 1e9

    # ---- the other operations (algorithmic bytes per op) ---
    def op_stats(prefix, bytes_fn):
        tt = bb = 0.0
        for c, a in zip(cases, packed):
            ts = times.get(f"{prefix}:{c['k']}:{int(c['signed'])}")
            if not ts:
                return None
            tt += sum(ts)
            bb += bytes_fn(c, a) * len(ts)
        return {"ms_per_sweep": round(tt / args.steps * 1e3, 3),
                "us_per_call": round(tt / args.steps / len(cases) * 1e6, 2),
                "alg_gbs": round(bb / tt / 1e9, 1)}

    ops = {"matvec": {"ms_per_sweep": round(tot_t / len(phases) * 1e3, 3),
                      "alg_gbs": round(value, 1)}}
    ops["compress"] = op_stats("compress", lambda c, a: 16 * n * n + 8 * a.words)
    if not args.profile:
        ops["add"] = op_stats("add", lambda c, a: 8 * (a.words + c["B"].words + c["sum"].words))
        ops["scale"] = op_stats("scale", lambda c, a: 8 * (a.words + c["scaled"].words))
        ops["decompress"] = op_stats("decompress", lambda c, a: 8 * a.words + 8 * n * n)
        ops["get_1000"] = op_stats("get", lambda c, a: 1000 * 8)

    # ---- dense int32 comparison and HBM read probe -----------------------
    del dec
    for c in cases:
        c["dense"] = None
    torch.cuda.empty_cache()
    dense32 = torch.empty((n, n), dtype=torch.int32, device="cuda")
    ccm.fill_uniform(dense32, -(1 << 15), 1 << 15, W.seed_for(2, 4), 0)
    copies32 = [dense32]
    for _ in range(1):
        copies32.append(dense32.clone())
    for i in range(3):
        bench_lib.ccmb_dense_matvec_i32(ctypes.c_void_p(copies32[i % 2].data_ptr()), n, n,
                                        ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(y.data_ptr()), sp)
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        bench_lib.ccmb_dense_matvec_i32(ctypes.c_void_p(copies32[i % 2].data_ptr()), n, n,
                                        ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(y.data_ptr()), sp)
    e1.record()
    torch.cuda.synchronize()
    td = e0.elapsed_time(e1) * 1e-3 / reps
    dense_i32 = {"matvec_us": round(td * 1e6, 2), "gelem_s": round(n * n / td / 1e9, 1),
                 "gbs": round(4 * n * n / td / 1e9, 1)}
    del copies32, dense32
    torch.cuda.empty_cache()

    # practical HBM read peak: a grid-stride 16-byte read of 1 GiB slices of a
    # 4 GiB buffer (each read leaves the 256 MB cache), over several grid
    # sizes; the best is reported
    big = torch.empty(4 << 30, dtype=torch.uint8, device="cuda")
    big.fill_(1)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    gib = 1 << 30
    read_by_grid = {}
    for grid in (1024, 2048, 4096, 8192):
        def rd(i, grid=grid):
            bench_lib.ccmb_read_bytes(ctypes.c_void_p(big.data_ptr() + (i % 4) * gib), gib,
                                      ctypes.c_void_p(sink.data_ptr()), grid, sp)
        for i in range(2):
            rd(i)
        e0.record()
        for i in range(8):
            rd(i)
        e1.record()
        torch.cuda.synchronize()
        read_by_grid[grid] = round(gib / (e0.elapsed_time(e1) * 1e-3 / 8) / 1e9, 1)
    read_peak = max(read_by_grid.values())
    # int8 matrix-unit peak: 4 waves per SIMD of back-to-back MFMA chains
    waves, iters = 4 * 4 * 256, 2048
    bench_lib.ccmb_mfma_i8_peak(waves, 64, ctypes.c_void_p(sink.data_ptr()), sp)
    e0.record()
    bench_lib.ccmb_mfma_i8_peak(waves, iters, ctypes.c_void_p(sink.data_ptr()), sp)
    e1.record()
    torch.cuda.synchronize()
    i8_peak = 4.0 * 65536 * iters * waves / (e0.elapsed_time(e1) * 1e-3) / 1e12
    # plain copy of known size (calibrates the FETCH_SIZE / WRITE_SIZE counters)
    half = big[: 1 << 30]
    big[2 << 30: 3 << 30].copy_(half)
    torch.cuda.synchronize()
    del big, half

    sweep_t = tot_t / len(phases)
    result = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic (seeded SplitMix64, generated on device, resident in HBM)",
        "config": {"workload": f"bandwidth sweep: {n}x{n}, k in {list(W.SWEEP_WIDTHS)}, "
                               "unsigned and signed, int32 x in [-2^15, 2^15)",
                   "rows": n, "cols": n, "matrices": len(cases),
                   "step": "compress, matvec, add, scale(7), decompress, 1000 gets; "
                           "all twelve matrices" if not args.profile else "compress, matvec"},
        "roofline": {"bound": "hbm", "achieved": round(value, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(value / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(),
                     "kernel": "matvec (one launch per sweep matrix)",
                     "alg_bytes_per_launch": round(sum(p["packed_bytes"] for p in per_width) /
                                                   len(per_width)),
                     "alg_bytes": "8*W packed bytes of A per launch (x and y not counted)"},
        "per_width": per_width,
        "ops": ops,
        "gelem_s_packed": round(len(per_width) * n * n / sweep_t / 1e9, 1),
        "dense_i32": dense_i32,
        "hbm_read_probe_gbs": round(read_peak, 1),
        "hbm_read_probe_by_grid": read_by_grid,
        "roofline_practical": {"hbm_read_gbs": round(read_peak, 1),
                               "frac": round(value / read_peak, 4),
                               "i8_mfma_tops": round(i8_peak, 1),
                               "i8_mfma_spec_tops": 5000.0},
    }

    log("dense int32 and read probe done")
    if not args.no_extras and not args.profile:
        from bench_extras import run_extras
        result["extras"] = run_extras(torch, ccm, log, i8_peak_measured=i8_peak)

    if not args.no_cpu_baseline and not args.profile:
        log("extras done; timing the oracle")
        result["cpu_baseline"] = cpu_baseline(W)

    print(json.dumps(result), flush=True)


def matvec_only(args, torch, W, ccm):
    """Matvec sweeps alone, for hardware-counter runs (one kernel per width)."""
    n = args.n
    mats = []
    x_spec = None
    for k in W.SWEEP_WIDTHS:
        for signed in (False, True):
            a_s, _, x_spec, _ = W.sweep(k, signed, n)
            mats.append(ccm.generate(n, n, a_s.lo, a_s.hi, a_s.seed, a_s.stream))
    x = torch.empty(n, dtype=torch.int32, device="cuda")
    ccm.fill_uniform(x, x_spec.lo, x_spec.hi, x_spec.seed, x_spec.stream)
    y = torch.empty(n, dtype=torch.int64, device="cuda")
    for _ in range(args.warmup + args.steps):
        for m in mats:
            ccm.matvec(m, x, y)
    src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"matvec_only": True, "matrices": len(mats),
                      "packed_bytes": [8 * m.words for m in mats]}), flush=True)


def cpu_baseline(W, rows=192, vlb_rows=32):
    """The oracle on the host cores, on the first `rows` rows of each of the
    twelve sweep matrices: the step's operations (compress A and B, matvec,
    add, scale by 7, decompress), each timed on one thread and on all cores.
    All cores: the sample's rows are split into one chunk per core and the
    oracle runs on the chunks from a thread pool (its calls release the
    interpreter lock); its own OpenMP loops are held to one thread throughout.
    value = the oracle's packed-matvec GB/s on all cores."""
    import ctypes.util
    from concurrent.futures import ThreadPoolExecutor


    import oracle
    cores = oracle.threads()
    gomp = ctypes.CDLL(ctypes.util.find_library("gomp") or "libgomp.so.1")
    gomp.omp_set_num_threads(1)
    samples = []
    for k in W.SWEEP_WIDTHS:
        for signed in (False, True):
            a_s, b_s, x_s, s = W.sweep(k, signed)
            samples.append((a_s.rows_slice(0, rows), b_s.rows_slice(0, rows), x_s.dense(), s))

    def run_ops(part):
        """part: list of (A rows, B rows, x, s); returns seconds per op."""
        t = dict.fromkeys(("compress", "matvec", "add", "scale", "decompress"), 0.0)
        for A, B, xv, s in part:
            t0 = time.perf_counter()
            pa, pb = oracle.compress(A), oracle.compress(B)
            t1 = time.perf_counter()
            oracle.matvec(pa, xv)
            t2 = time.perf_counter()
            oracle.add(pa, pb)
            t3 = time.perf_counter()
            oracle.scale(pa, s)
            t4 = time.perf_counter()
            oracle.decompress(pa)
            t5 = time.perf_counter()
            for key, dt in (("compress", t1 - t0), ("matvec", t2 - t1), ("add", t3 - t2),
                            ("scale", t4 - t3), ("decompress", t5 - t4)):
                t[key] += dt
        return t

    w0 = time.perf_counter()
    one = run_ops(samples)
    t_one = time.perf_counter() - w0
    chunk = -(-rows // cores)
    parts = [[(A[r:r + chunk], B[r:r + chunk], xv, s) for A, B, xv, s in samples]
             for r in range(0, rows, chunk)]
    packed = [[(oracle.compress(A), oracle.compress(B), xv, s) for A, B, xv, s in p]
              for p in parts]

    def all_cores(fn):
        """Wall time of fn(i) for every chunk i, one pool thread per chunk."""
        w = time.perf_counter()
        with ThreadPoolExecutor(len(parts)) as ex:
            list(ex.map(fn, range(len(parts))))
        return time.perf_counter() - w

    alls = {
        "compress": all_cores(lambda i: [(oracle.compress(A), oracle.compress(B))
                                         for A, B, _, _ in parts[i]]),
        "matvec": all_cores(lambda i: [oracle.matvec(pa, xv) for pa, _, xv, _ in packed[i]]),
        "add": all_cores(lambda i: [oracle.add(pa, pb) for pa, pb, _, _ in packed[i]]),
        "scale": all_cores(lambda i: [oracle.scale(pa, s) for pa, _, _, s in packed[i]]),
        "decompress": all_cores(lambda i: [oracle.decompress(pa) for pa, _, _, _ in packed[i]]),
    }
    t_all = sum(alls.values())
    n = rows * samples[0][0].shape[1]
    a_bytes = sum(n * oracle.width(int(A.min()), int(A.max()))[0] / 8 for A, _, _, _ in samples)
    per_op = {}
    for key in ("compress", "matvec", "add", "scale", "decompress"):
        per_op[key] = {"one_thread_s": round(one[key], 4), "all_cores_s": round(alls[key], 4),
                       "one_thread_melem_s": round(12 * n / one[key] / 1e6, 2),
                       "all_cores_melem_s": round(12 * n / alls[key] / 1e6, 2)}
    # Method 2: the oracle's matvec on the first rows of each Beta workload
    # (each row compressed on its own; its y entry is the same), one thread
    vlb = {}
    for name in W.VLB_BETAS:
        spec, x_s = W.vlb_sweep(name)
        xv = x_s.dense()
        pk = [oracle.vlb_compress(spec.rows_slice(r, r + 1)) for r in range(vlb_rows)]
        t0 = time.perf_counter()
        for p in pk:
            oracle.vlb_matvec(p, xv)
        dt = time.perf_counter() - t0
        vlb[name] = {"gelem_s": round(vlb_rows * spec.cols / dt / 1e9, 5),
                     "gb_s": round(sum(p.nbits for p in pk) / 8 / dt / 1e9, 5)}
    gomp.omp_set_num_threads(cores)
    return {"value": round(a_bytes / alls["matvec"] / 1e9, 4), "unit": "GB/s",
            "cores": cores, "kind": "oracle",
            "value_one_thread": round(a_bytes / one["matvec"] / 1e9, 4),
            "per_op": per_op,
            "step_one_thread_s": round(t_one, 2), "step_all_cores_s": round(t_all, 2),
            "vlb_matvec": vlb, "vlb_sample": f"rows 0..{vlb_rows - 1} of each 16384 x 16384 "
                                             "Beta workload, one thread",
            "sample": f"rows 0..{rows - 1} of each of the 12 sweep matrices ({12 * rows} x 16384 "
                      "elements): compress A and B, matvec, add, scale, decompress, each on one "
                      "thread and on all cores (rows split over a thread pool); value = packed "
                      "bytes of A over the oracle's all-cores matvec time"}


if __name__ == "__main__":
    main()
