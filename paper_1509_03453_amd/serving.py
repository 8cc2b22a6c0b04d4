"""Continuous-batching search server over several resident indexes.

Requests (a batch of 1..4096 queries against one named index) arrive over
time.  The server keeps every index resident on the device and runs a host
loop that

* moves requests whose arrival time has come into a per-index queue;
* retires launches whose completion event has fired, releasing their slot
  and their device memory;
* admits queued work while a slot is free AND the device memory it needs
  (the library's workspace for that batch, staging for the queries and the
  outputs) fits both in the free HBM above a reserve and in the pool cap;
* packs the oldest queued requests of one index into a micro-batch of at most
  ``max_batch`` queries (whole requests only; one request larger than the cap
  goes alone) and launches one ``os_ann_search_ex`` on that slot's stream,
  by default as a replay of the library's hipGraph for the batch's shape
  class (``OS_ANN_FLAG_GRAPH``: one graph per slot stream and class, all
  captured during ``warmup``).

So requests arriving while others are on the GPU start as soon as a slot and
memory free up, and their kernels overlap on the device.  Latency is the
completion event of a request's batch (device clock) minus its scheduled
arrival (host clock) moved onto the device clock: while the device is idle,
before and after the run, events are recorded at known host times and their
device times give the offset between the two clocks; the run reports that
offset's spread and drift, which bound the error of every latency.

The search itself (hash, probe, screen, re-rank) is entirely in the HIP
library: this module only schedules calls to it.  A query's result does not
depend on which other queries share its launch (every accumulation order is
fixed per (query, candidate) pair and the candidate lists are ordered by a
total order), so a request gets the same answer alone and in the mix.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Sequence

import numpy as np
import torch

from . import binding as B

__all__ = ["Request", "ResidentIndex", "Server", "pack_batch", "admissible", "latency_stats", "choose_mode",
           "load_sweep", "graph_classes"]


@dataclasses.dataclass
class Request:
    """One client request: ``queries`` (device, rows of the index's query type) for index ``index``."""
    rid: int
    index: str
    queries: torch.Tensor
    arrival: float                       # seconds after the run starts
    out_idx: torch.Tensor | None = None  # filled on completion (device views)
    out_dist: torch.Tensor | None = None
    launched: float | None = None        # host seconds when its batch was launched
    done: float | None = None            # device seconds of its batch's completion event
    batch_id: int | None = None
    lag: float | None = None             # host seconds from scheduled arrival to queueing
    offset: float | None = None          # device minus host clock (seconds) of the run

    @property
    def n(self) -> int:
        return int(self.queries.shape[0])

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - (self.arrival + self.offset)


@dataclasses.dataclass
class ResidentIndex:
    """A built index kept on the device with its serving parameters."""
    name: str
    index: B.Index
    budget: int
    mode: int = B.OS_ANN_MODE_TILED
    rerank_r: int = 8

    def workspace(self, q: int) -> int:
        return self.index.workspace_bytes(q, self.budget, self.mode, self.rerank_r)


def choose_mode(index: B.Index, queries: torch.Tensor, budget: int, rerank_r: int = 8, reps: int = 3) -> int:
    """The faster search mode for this index and budget, timed on ``queries``.

    Both modes visit the same candidates; the matrix-core screening pays off
    when queries probe many cones, the plain scan when they probe few."""
    best, best_ms = B.OS_ANN_MODE_FP32, None
    for mode in (B.OS_ANN_MODE_FP32, B.OS_ANN_MODE_TILED):
        index.search(queries, budget, mode=mode, rerank_r=rerank_r)  # warm-up (and split choice)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            index.search(queries, budget, mode=mode, rerank_r=rerank_r)
        t1.record()
        t1.synchronize()
        ms = t0.elapsed_time(t1) / reps
        if best_ms is None or ms < best_ms:
            best, best_ms = mode, ms
    return best


# ---------------------------------------------------------------------------
# scheduling policy (pure functions, host only)
# ---------------------------------------------------------------------------
def pack_batch(queue: Sequence[int], max_batch: int) -> int:
    """How many requests, from the head of ``queue`` (their query counts), go into one launch.

    Whole requests are taken in arrival order while the total stays within
    ``max_batch``; the head request is always taken, even when it alone is
    larger than the cap."""
    total, k = 0, 0
    for n in queue:
        if k > 0 and total + n > max_batch:
            break
        total += n
        k += 1
    return k


def admissible(need: int, free_hbm: int, reserve: int, in_flight: int, pool_cap: int) -> bool:
    """A launch needing ``need`` device bytes may start: it fits above the reserve and under the cap."""
    return need <= free_hbm - reserve and in_flight + need <= pool_cap


def latency_stats(lat: Sequence[float]) -> dict:
    """p50 / p99 / mean / max of latencies in seconds, reported in milliseconds."""
    a = np.asarray(lat, dtype=np.float64) * 1e3
    if a.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None, "max_ms": None}
    return {"p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean()), "max_ms": float(a.max())}


def clock_offsets(base, t0: float, device, n: int = 16) -> np.ndarray:
    """Device-minus-host clock offsets (seconds): with the device idle, an
    event is recorded at a known host time (seconds after ``t0``) and its
    device time read relative to ``base``; the event completes a little
    after the host enqueues it, so each sample is the offset plus that
    submission delay, and their spread shows the delay's variation."""
    stream = torch.cuda.current_stream(device)
    out = []
    for _ in range(n):
        ev = torch.cuda.Event(enable_timing=True)
        h = time.perf_counter() - t0
        ev.record(stream)
        ev.synchronize()
        out.append(base.elapsed_time(ev) * 1e-3 - h)
    return np.asarray(out)


def pick_index(queues: dict[str, collections.deque]) -> str | None:
    """The index whose oldest queued request arrived first (first come, first served)."""
    best, t = None, None
    for name, q in queues.items():
        if q and (t is None or q[0].arrival < t):
            best, t = name, q[0].arrival
    return best


def graph_classes(max_q: int) -> list[int]:
    """The query counts of the library's graph shape classes up to ``max_q``
    (OS_ANN_FLAG_GRAPH: Q rounded up to one of eight steps per octave; 8 and
    16 below that), ascending; the last one covers ``max_q``."""
    out, q = [], 1
    while True:
        if q <= 8:
            c = 8
        elif q <= 16:
            c = 16
        else:
            k = (q - 1).bit_length() - 1  # 2^k < q <= 2^(k+1)
            step = (1 << k) // 8
            c = (q + step - 1) // step * step
        out.append(c)
        if c >= max_q:
            return out
        q = c + 1


# ---------------------------------------------------------------------------
# the server
# ---------------------------------------------------------------------------
class _Slot:
    def __init__(self, device):
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.event = torch.cuda.Event(enable_timing=True)
        self.reqs: list[Request] = []
        self.hold: tuple = ()
        self.bytes = 0
        self.busy = False
        self.ws = None  # the slot's search workspace; grows to the largest launch, then is reused


class Server:
    """Serve requests against resident indexes with continuous batching on ``slots`` streams.

    ``pool_cap_bytes`` bounds the device memory held by launches in flight;
    ``reserve_bytes`` is the free HBM left untouched for everything else."""

    def __init__(self, indexes: Sequence[ResidentIndex], slots: int = 4, max_batch: int = 8192,
                 pool_cap_bytes: int = 4 << 30, reserve_bytes: int = 1 << 30,
                 device: torch.device | str = "cuda:0",
                 free_hbm: Callable[[], int] | None = None, graphs: bool = True):
        if slots < 1 or max_batch < 1:
            raise ValueError("slots and max_batch must be positive")
        self.indexes = {r.name: r for r in indexes}
        self.device = torch.device(device)
        self.max_batch = int(max_batch)
        self.pool_cap = int(pool_cap_bytes)
        self.reserve = int(reserve_bytes)
        self.slots = [_Slot(self.device) for _ in range(slots)]
        self._free_hbm = free_hbm or self._device_free
        self.in_flight = 0
        self.n_batches = 0
        self.peak_in_flight = 0
        self.max_concurrent = 0
        self.graphs = bool(graphs)

    def _device_free(self) -> int:
        free, _ = torch.cuda.mem_get_info(self.device)
        # blocks the caching allocator holds but does not use are free to us too
        cached = torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
        return int(free + cached)

    def need_bytes(self, ix: ResidentIndex, q: int, qbytes_per_row: int) -> int:
        return ix.workspace(q) + q * (qbytes_per_row + 8 + 4)

    def warmup(self, samples: dict[str, torch.Tensor]) -> None:
        """Runs every index once per power-of-two batch size up to ``max_batch``, on queries drawn
        from its own distribution (``samples[name]``, at least ``max_batch`` rows), so that the
        library's per-size choices are made and cached before requests are timed."""
        for name, ix in self.indexes.items():
            x = samples[name]
            q = 1
            while True:
                q = min(q, self.max_batch, x.shape[0])
                ix.index.search(x[:q], ix.budget, mode=ix.mode, rerank_r=ix.rerank_r)
                if q >= min(self.max_batch, x.shape[0]):
                    break
                q *= 2
        if self.graphs:
            # every (slot, shape class) graph captured now, largest class first so that each
            # slot's graph buffers are sized once
            for name, ix in self.indexes.items():
                x = samples[name]
                for q in reversed(graph_classes(min(self.max_batch, x.shape[0]))):
                    for s in self.slots:
                        with torch.cuda.stream(s.stream):
                            B.os_ann_search_ex(ix.index.handle, x[:q], ix.budget, mode=ix.mode, stream=s.stream,
                                               rerank_r=ix.rerank_r, want_ncand=False, flags=B.OS_ANN_FLAG_GRAPH)
            torch.cuda.synchronize(self.device)
            return
        # every slot's workspace sized for the largest launch, so timed launches allocate none
        need = max(ix.workspace(self.max_batch) for ix in self.indexes.values())
        for s in self.slots:
            with torch.cuda.stream(s.stream):
                s.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)

    def _launch(self, slot: _Slot, ix: ResidentIndex, reqs: list[Request], need: int, now: float) -> None:
        q_total = sum(r.n for r in reqs)
        with torch.cuda.stream(slot.stream):
            qs = reqs[0].queries if len(reqs) == 1 else torch.cat([r.queries for r in reqs])
            oi = torch.empty(q_total, dtype=torch.int64, device=self.device)
            od = torch.empty(q_total, dtype=torch.float32, device=self.device)
            if self.graphs:  # the library keeps the graph's buffers per slot stream
                ws = None
                B.os_ann_search_ex(ix.index.handle, qs, ix.budget, mode=ix.mode, stream=slot.stream,
                                   rerank_r=ix.rerank_r, out_idx=oi, out_dist=od, want_ncand=False,
                                   flags=B.OS_ANN_FLAG_GRAPH)
            else:
                wsb = ix.workspace(q_total)
                if slot.ws is None or slot.ws.numel() < wsb:
                    slot.ws = None  # the old buffer is idle: this slot's previous launch has retired
                    slot.ws = torch.empty(wsb, dtype=torch.uint8, device=self.device)
                ws = slot.ws
                B.os_ann_search_ex(ix.index.handle, qs, ix.budget, mode=ix.mode, stream=slot.stream,
                                   workspace=ws, rerank_r=ix.rerank_r, out_idx=oi, out_dist=od,
                                   want_ncand=False)
            slot.event.record(slot.stream)
        off = 0
        for r in reqs:
            r.out_idx, r.out_dist = oi[off:off + r.n], od[off:off + r.n]
            r.launched, r.batch_id = now, self.n_batches
            off += r.n
        slot.reqs, slot.hold, slot.bytes, slot.busy = reqs, (qs, ws, oi, od), need, True
        self.in_flight += need
        self.n_batches += 1
        self.peak_in_flight = max(self.peak_in_flight, self.in_flight)
        self.max_concurrent = max(self.max_concurrent, sum(s.busy for s in self.slots))

    def run(self, requests: Sequence[Request], max_seconds: float = 600.0) -> dict:
        """Serves ``requests`` (arrival times relative to the start) and returns throughput and latency."""
        for r in requests:
            if r.index not in self.indexes:
                raise KeyError(f"request {r.rid} names unknown index {r.index!r}")
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queues = {name: collections.deque() for name in self.indexes}
        base = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(self.device)
        base.record(torch.cuda.current_stream(self.device))
        base.synchronize()
        t0 = time.perf_counter()
        before = clock_offsets(base, t0, self.device)
        finished: list[Request] = []
        while pending or any(queues.values()) or any(s.busy for s in self.slots):
            now = time.perf_counter() - t0
            if now > max_seconds:
                raise TimeoutError(f"serving run exceeded {max_seconds} s")
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                r.lag = now - r.arrival
                queues[r.index].append(r)
            for s in self.slots:  # retire
                if s.busy and s.event.query():
                    t_done = base.elapsed_time(s.event) * 1e-3
                    for r in s.reqs:
                        r.done = t_done
                    finished.extend(s.reqs)
                    self.in_flight -= s.bytes
                    s.reqs, s.hold, s.bytes, s.busy = [], (), 0, False
            progressed = False
            for s in self.slots:  # admit
                if s.busy:
                    continue
                name = pick_index(queues)
                if name is None:
                    break
                ix, q = self.indexes[name], queues[name]
                k = pack_batch([r.n for r in q], self.max_batch)
                reqs = [q[i] for i in range(k)]
                row_bytes = reqs[0].queries.element_size() * reqs[0].queries.shape[1]
                need = self.need_bytes(ix, sum(r.n for r in reqs), row_bytes)
                if not admissible(need, self._free_hbm(), self.reserve, self.in_flight, self.pool_cap):
                    if self.in_flight == 0:
                        raise MemoryError(f"request {reqs[0].rid} needs {need} B; pool cap or free HBM too small")
                    break
                for _ in range(k):
                    q.popleft()
                self._launch(s, ix, reqs, need, now)
                progressed = True
            if not progressed:
                time.sleep(5e-5)
        wall = time.perf_counter() - t0
        torch.cuda.synchronize(self.device)
        after = clock_offsets(base, t0, self.device)
        offset = float(np.median(before))
        for r in finished:
            r.offset = offset
        n_q = sum(r.n for r in finished)
        span = max(r.done for r in finished) - min(r.arrival for r in finished) if finished else 0.0
        out = {"requests": len(finished), "queries": n_q, "batches": self.n_batches,
               "qps": n_q / span if span > 0 else None, "span_s": span, "wall_s": wall,
               "max_concurrent_launches": self.max_concurrent, "peak_in_flight_bytes": self.peak_in_flight}
        out.update(latency_stats([r.latency for r in finished]))
        lag = np.asarray([r.lag for r in finished]) * 1e3
        out["arrival_lag_ms"] = {"p50": float(np.percentile(lag, 50)), "max": float(lag.max())} if lag.size else None
        out["clock_offset_us"] = {"before_median": offset * 1e6,
                                  "before_spread": float(np.ptp(before)) * 1e6,
                                  "after_median": float(np.median(after)) * 1e6,
                                  "drift": float(np.median(after) - offset) * 1e6}
        return out


def load_sweep(server: "Server", make_requests: Callable[[float], list], fractions=(0.5, 0.8, 0.95),
               warmup_requests: int = 100, saturation_requests: int = 600, max_seconds: float = 300.0) -> dict:
    """Saturation rate, then Poisson load points at fractions of it.

    ``make_requests(rate)`` returns a fresh request list with arrivals at
    ``rate`` requests/s (rate = inf: every request at time 0).  The
    saturation rate is the request rate the server sustains with the first
    ``saturation_requests`` requests queued at once.  Each load point runs
    the whole list and reports throughput and latency over the requests
    after the first ``warmup_requests``.  Returns the summary and the
    requests of the last load point (with their results)."""
    sat_reqs = make_requests(float("inf"))[:saturation_requests]
    st = server.run(sat_reqs, max_seconds=max_seconds)
    sat_rate = st["requests"] / st["span_s"]
    out = {"saturation": {"req_per_s": sat_rate, "qps": st["qps"], "requests": st["requests"]}, "points": []}
    reqs = []
    for f in fractions:
        reqs = make_requests(f * sat_rate)
        server.run(reqs, max_seconds=max_seconds)
        meas = reqs[warmup_requests:]
        t_first = min(r.arrival for r in meas)
        t_last = max(r.done for r in meas)
        pt = {"fraction": f, "offered_req_per_s": f * sat_rate, "measured_requests": len(meas),
              "qps": sum(r.n for r in meas) / (t_last - t_first),
              "req_per_s": len(meas) / (t_last - t_first)}
        pt.update(latency_stats([r.latency for r in meas]))
        out["points"].append(pt)
    return out, reqs
