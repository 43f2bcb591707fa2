"""Serving loop over a pool of compressed matrices resident in HBM.

Requests (matvec with an int32 x, or matmul with a small compressed B) arrive
over time.  The loop runs continuous batching on a few HIP streams:

* admission: a request is admitted when a slot is free (at most `max_inflight`
  requests admitted and not finished) and its memory footprint (x and y, or B,
  the result at its bound width and the matmul scratch) fits in the arena left
  after the pool;
* every admitted matvec not yet launched goes into the next batched launch
  (one persistent kernel over all of them, ccm_batch_matvec_dyn) on the next
  free stream -- matrices wider than the batched kernel's x staging take the
  single-matrix kernel in the same launch; a matmul runs on a free stream of
  its own (ccm_matmul_async: its result width is decided on the device, and
  its header fields are read back only once the launch has completed);
* nothing in the loop waits for the device: launches are enqueued, and
  completion is polled;
* launches on different streams overlap on the device; requests that arrive
  while others run are admitted as slots and memory free up and join the next
  launch;
* completion is read from a GPU event per launch; latency is completion time
  minus arrival time, both on the run's clock (the GPU timestamps are taken
  relative to an event recorded when the run starts);
* Python's cyclic garbage collector is paused for the run (a full collection
  over a process that has imported torch can hold the loop for tens of
  milliseconds); `max_loop_gap_ms` reports the longest time between two
  passes of the loop, so a host-side stall shows in the statistics;
* the loop allocates no device memory: every result buffer (y of each
  matvec, the payload and workspace of each matmul) and one matmul scratch
  per stream are carved out of a few tensors before the first request, so
  that no block the caching allocator does not hold yet can mean a hipMalloc
  inside the loop (a run that still allocated there once showed a 6 ms
  stall of the loop at 95 % load; its cause was not isolated).
"""
from __future__ import annotations

import collections
import gc
import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import (CMatrix, Pending, generate, lib, matmul_async, matmul_capacity,
               matmul_scratch_bytes, matvec)
from .batch import BATCH_MAX_COLS, DynBatch


@dataclass
class Request:
    rid: int
    kind: str  # "mv" or "mm"
    mat: int  # index into the pool
    arrival: float  # seconds after the start of the run
    x: torch.Tensor | None = None  # matvec input (int32)
    b: CMatrix | None = None  # matmul right operand
    footprint: int = 0
    y: torch.Tensor | None = None  # matvec result
    c: CMatrix | None = None  # matmul result
    pending: Pending | None = None  # matmul result while in flight
    buf: torch.Tensor | None = None  # y (matvec) or the result payload (matmul), preassigned
    ws: torch.Tensor | None = None  # matmul result workspace, preassigned
    done: float = math.nan  # completion, seconds after the start of the run
    launch: int = -1  # id of the launch that served it


@dataclass
class _Launch:
    lid: int
    stream_idx: int
    start: torch.cuda.Event
    event: torch.cuda.Event
    requests: list
    hosts: list = field(default_factory=list)  # pinned result buffers to hand back


def request_footprint(req: Request, pool) -> int:
    """Device bytes a request holds while in flight: x and y, or B, the
    result at the width the operand headers bound, the matmul scratch and
    the result's workspace."""
    a = pool[req.mat]
    if req.kind == "mv":
        return 4 * a.cols + 8 * a.rows
    b = req.b
    return (b.payload.numel() + matmul_capacity(a, b) + matmul_scratch_bytes(a, b) +
            int(lib.ccm_async_ws_bytes()))


class Server:
    def __init__(self, pool, arena_bytes: int, streams: int = 4, max_inflight: int = 256,
                 max_batch: int = 512):
        self.pool = pool
        self.arena = int(arena_bytes)
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.dyn = [DynBatch(max_mats=max_batch, max_items=1 << 17, slots=4)
                    for _ in range(streams)]
        # pinned 64-byte buffers receiving matmul results' header fields
        self._hosts_mem = torch.empty((max_inflight, 64), dtype=torch.uint8, pin_memory=True)
        self._hosts = [self._hosts_mem[i] for i in range(max_inflight)]

    def close(self):
        for d in self.dyn:
            d.close()

    def run(self, requests, poll_sleep: float = 0.0):
        """Serves `requests` (sorted by arrival); returns summary statistics.
        Each request's result is left in req.y / req.c."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            r.footprint = request_footprint(r, self.pool)
            if r.footprint > self.arena:
                raise ValueError(f"request {r.rid} needs {r.footprint} bytes, arena {self.arena}")
        scratch = self._prepare(reqs)
        torch.cuda.synchronize()
        gc_was_enabled = gc.isenabled()
        gc.collect()
        gc.disable()
        try:
            return self._loop(reqs, poll_sleep, scratch)
        finally:
            if gc_was_enabled:
                gc.enable()

    def _prepare(self, reqs):
        """Device buffers of the whole run, assigned before the loop starts:
        views of one int64 tensor for the matvec results, of one byte tensor
        (256-byte aligned slices) for the matmul payloads and workspaces, and
        one scratch per stream (a stream runs its matmuls in order, so each
        reuses it).  Returns the per-stream scratch list."""
        dev = torch.device("cuda")
        mv = [r for r in reqs if r.kind == "mv"]
        mm = [r for r in reqs if r.kind != "mv"]
        rows = [self.pool[r.mat].rows for r in mv]
        ys = torch.empty(max(1, sum(rows)), dtype=torch.int64, device=dev)
        off = 0
        for r, n in zip(mv, rows):
            r.buf = ys[off:off + n]
            off += n
        def up(n):
            return (n + 255) // 256 * 256
        wsb = int(lib.ccm_async_ws_bytes())
        caps = [matmul_capacity(self.pool[r.mat], r.b) for r in mm]
        need = max([matmul_scratch_bytes(self.pool[r.mat], r.b) for r in mm], default=0)
        blob = torch.empty(max(1, sum(up(c) + up(wsb) for c in caps)), dtype=torch.uint8,
                           device=dev)
        off = 0
        for r, c in zip(mm, caps):
            r.buf = blob[off:off + c]
            off += up(c)
            r.ws = blob[off:off + wsb]
            off += up(wsb)
        return [torch.empty(max(1, need), dtype=torch.uint8, device=dev)
                for _ in self.streams]

    def _loop(self, reqs, poll_sleep, scratch):
        waiting = collections.deque()
        pending_mv, pending_mm = [], []
        inflight: list[_Launch] = []
        free_streams = list(range(len(self.streams)))
        used_bytes = 0
        admitted = 0
        lid = 0
        nxt = 0
        n = len(reqs)
        finished = 0
        launches = []
        done_launches = []
        max_inflight_seen = 0
        max_gap = 0.0
        start_evt = torch.cuda.Event(enable_timing=True)
        start_evt.record()
        t0 = time.perf_counter()
        last = 0.0
        while finished < n:
            now = time.perf_counter() - t0
            max_gap = max(max_gap, now - last)
            last = now
            while nxt < n and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            # completions (polled; the header fields of a matmul result are
            # on the host once its launch's event has completed)
            still = []
            for L in inflight:
                if L.event.query():
                    t_done = start_evt.elapsed_time(L.event) * 1e-3
                    for r in L.requests:
                        if r.pending is not None:
                            r.c = r.pending.get()
                            r.pending = None
                        r.done = t_done
                        used_bytes -= r.footprint
                        admitted -= 1
                        finished += 1
                    free_streams.append(L.stream_idx)
                    self._hosts.extend(L.hosts)
                    done_launches.append(L)
                else:
                    still.append(L)
            inflight = still
            # admission
            while waiting and admitted < self.max_inflight and \
                    used_bytes + waiting[0].footprint <= self.arena:
                r = waiting.popleft()
                used_bytes += r.footprint
                admitted += 1
                (pending_mv if r.kind == "mv" else pending_mm).append(r)
            # launches
            while free_streams and (pending_mv or pending_mm):
                si = free_streams.pop(0)
                stream = self.streams[si]
                L = _Launch(lid, si, torch.cuda.Event(enable_timing=True),
                            torch.cuda.Event(enable_timing=True), [])
                with torch.cuda.stream(stream):
                    L.start.record(stream)
                    if pending_mm and (not pending_mv or len(pending_mm) * 8 >= len(pending_mv)):
                        r = pending_mm.pop(0)
                        host = self._hosts.pop()
                        r.pending = matmul_async(self.pool[r.mat], r.b, scratch=scratch[si],
                                                 ws=r.ws, payload=r.buf, host=host,
                                                 stream=stream)
                        L.requests.append(r)
                        L.hosts.append(host)
                    else:
                        group = pending_mv[: self.max_batch]
                        del pending_mv[: len(group)]
                        narrow = []
                        for r in group:
                            a = self.pool[r.mat]
                            r.y = r.buf
                            if a.cols <= BATCH_MAX_COLS:
                                narrow.append(r)
                            else:
                                matvec(a, r.x, r.y, stream=stream)
                        if narrow:
                            self.dyn[si].matvec([self.pool[r.mat] for r in narrow],
                                                [r.x for r in narrow], [r.y for r in narrow],
                                                stream=stream)
                        L.requests.extend(group)
                    L.event.record(stream)
                for r in L.requests:
                    r.launch = lid
                inflight.append(L)
                max_inflight_seen = max(max_inflight_seen, len(inflight))
                launches.append(len(L.requests))
                lid += 1
            if poll_sleep:
                time.sleep(poll_sleep)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # launches whose device execution overlapped an earlier launch's, and
        # matmul launches that overlapped a matvec launch
        spans = sorted((start_evt.elapsed_time(L.start), start_evt.elapsed_time(L.event),
                        L.requests[0].kind) for L in done_launches)
        overlapped, end_max = 0, -math.inf
        for s0, s1, _ in spans:
            overlapped += s0 < end_max
            end_max = max(end_max, s1)
        mv_spans = [(s0, s1) for s0, s1, k in spans if k == "mv"]
        mm_with_mv = sum(any(a0 < s1 and s0 < a1 for a0, a1 in mv_spans)
                         for s0, s1, k in spans if k == "mm")
        lat = np.array([r.done - r.arrival for r in reqs])
        span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
        touched = sum(8 * self.pool[r.mat].words for r in reqs)
        return {"requests": n, "launches": lid,
                "mean_batch": round(float(np.mean(launches)), 2) if launches else 0.0,
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "mean_ms": round(float(lat.mean()) * 1e3, 3),
                "throughput_rps": round(n / span, 1),
                "throughput_gbs": round(touched / span / 1e9, 1),
                "max_launches_in_flight": max_inflight_seen,
                "overlapped_launches": int(overlapped),
                "mm_overlapping_mv": int(mm_with_mv),
                "max_loop_gap_ms": round(max_gap * 1e3, 3),
                "wall_s": round(wall, 4)}


def make_pool(specs):
    """Generates the pool on the device (no dense copies)."""
    return [generate(p.rows, p.cols, p.spec.lo, p.spec.hi, p.spec.seed, p.spec.stream)
            for p in specs]


# generator streams of the per-request inputs: x of request rid uses stream
# X_STREAM + rid, B uses B_STREAM + rid (same seed as the request mix)
X_STREAM = 1 << 20
B_STREAM = 1 << 21


def make_requests(pool, count: int, qps: float | None, seed: int, mm_frac: float = 0.1,
                  mm_max_elems: int = 1 << 20, first_rid: int = 0):
    """Seeded request mix: 90% matvec on a uniformly chosen pool matrix with
    int32 x in [-2^15, 2^15); 10% matmul of a pool matrix with <= 2^20
    elements by a compressed B (cols x n, n in [2, 64], signed, width 1..8).
    qps=None: every request arrives at t = 0 (saturation)."""
    from . import fill_uniform
    rng = np.random.default_rng(seed)
    small = [i for i, m in enumerate(pool) if m.rows * m.cols <= mm_max_elems]
    out = []
    t = 0.0
    for k in range(count):
        if qps:
            t += float(rng.exponential(1.0 / qps))
        rid = first_rid + k
        if small and rng.random() < mm_frac:
            mi = int(small[int(rng.integers(0, len(small)))])
            a = pool[mi]
            ncol = int(rng.integers(2, 65))
            bw = int(rng.integers(1, 9))
            lo, hi = -(1 << (bw - 1)), (1 << (bw - 1)) if bw > 1 else 1
            if bw == 1:
                lo, hi = -1, 1
            b = generate(a.cols, ncol, lo, hi, seed, B_STREAM + rid)
            out.append(Request(rid, "mm", mi, t, b=b))
        else:
            mi = int(rng.integers(0, len(pool)))
            x = torch.empty(pool[mi].cols, dtype=torch.int32, device="cuda")
            fill_uniform(x, -(1 << 15), 1 << 15, seed, X_STREAM + rid)
            out.append(Request(rid, "mv", mi, t, x=x))
    torch.cuda.synchronize()
    return out
