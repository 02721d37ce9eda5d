"""Online IMCE serving: edge-addition batches handled as they arrive.

Each session owns a device-resident incremental state (graph, clique count
and set hash) and a HIP stream of its own.  Requests (session, batch) enter a
pending queue with their arrival time.  The admission loop starts a request
when (a) its session has no batch in flight (batches of one stream are
causally ordered), (b) a slot is free, and (c) its memory estimate fits the
budget; admitted requests run concurrently on worker threads, one per slot,
each driving its session's stream, so their kernels overlap on the device.
As soon as a request finishes its slot and memory return and the next
eligible request is admitted: continuous batching across sessions.

Latency = completion - arrival (queueing included); p50/p99 by nearest rank.
"""

from __future__ import annotations

import math
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import ImceState, _torch


@dataclass
class Request:
    session: int
    seq: int
    src: np.ndarray
    dst: np.ndarray
    arrival: float = 0.0
    start: float = 0.0
    end: float = 0.0
    result: Optional[dict] = None
    error: Optional[str] = None

    @property
    def latency_ms(self) -> float:
        return (self.end - self.arrival) * 1e3


def nearest_rank(values: Sequence[float], q: float) -> float:
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, int(math.ceil(q / 100.0 * len(v))))
    return float(v[k - 1])


def estimate_bytes(rho: int) -> int:
    """Device memory a batch may add beyond its session's resident state:
    batch keys and sorts, edge subproblem tables and rows, clique buffers."""
    return 256 * 1024 + rho * 4096


class Server:
    def __init__(self, graphs: Sequence, slots: int = 4, mem_budget: Optional[int] = None, **launch):
        torch = _torch()
        self.torch = torch
        self.streams = [torch.cuda.Stream() for _ in graphs]
        self.states = []
        for g, st in zip(graphs, self.streams):
            with torch.cuda.stream(st):
                self.states.append(ImceState(g, stream=st, **launch))
        torch.cuda.synchronize()
        self.slots = slots
        if mem_budget is None:
            free, _total = torch.cuda.mem_get_info()
            mem_budget = int(free * 0.5)
        self.mem_budget = mem_budget
        self.lock = threading.Condition()
        self.pending: List[Request] = []
        self.busy_sessions = set()
        self.in_flight = 0
        self.mem_in_use = 0
        self.done: List[Request] = []
        self.max_in_flight = 0
        self.max_overlap_sessions = 0
        self.on_done = None  # called with each finished request, under the lock

    def close(self):
        for s in self.states:
            s.close()

    def submit(self, req: Request):
        with self.lock:
            req.arrival = time.perf_counter() if req.arrival == 0.0 else req.arrival
            self.pending.append(req)
            self.lock.notify_all()

    def _eligible(self) -> Optional[Request]:
        # oldest pending request whose session is idle and whose estimate fits
        for i, r in enumerate(self.pending):
            if r.session in self.busy_sessions:
                continue
            need = estimate_bytes(len(r.src))
            if self.mem_in_use + need > self.mem_budget and self.in_flight > 0:
                continue
            # keep per-session order: no older pending request of the same session
            if any(p.session == r.session and p.seq < r.seq for p in self.pending[:i]):
                continue
            return self.pending.pop(i)
        return None

    def _run(self, req: Request):
        torch = self.torch
        st = self.states[req.session]
        try:
            with torch.cuda.stream(self.streams[req.session]):
                req.start = time.perf_counter()
                req.result = st.add(req.src, req.dst)
                req.end = time.perf_counter()
        except Exception as e:  # reported per request
            req.error = repr(e)
            req.end = time.perf_counter()
        with self.lock:
            self.busy_sessions.discard(req.session)
            self.in_flight -= 1
            self.mem_in_use -= estimate_bytes(len(req.src))
            self.done.append(req)
            if self.on_done is not None:
                self.on_done(req)
            self.lock.notify_all()

    def serve(self, total: int, poll_s: float = 0.0005):
        """Admits and runs requests until `total` have completed."""
        workers = []
        with self.lock:
            while len(self.done) < total:
                started = False
                while self.in_flight < self.slots:
                    r = self._eligible()
                    if r is None:
                        break
                    self.busy_sessions.add(r.session)
                    self.in_flight += 1
                    self.mem_in_use += estimate_bytes(len(r.src))
                    self.max_in_flight = max(self.max_in_flight, self.in_flight)
                    self.max_overlap_sessions = max(self.max_overlap_sessions, len(self.busy_sessions))
                    t = threading.Thread(target=self._run, args=(r,), daemon=True)
                    t.start()
                    workers.append(t)
                    started = True
                if not started:
                    self.lock.wait(timeout=poll_s)
        for t in workers:
            t.join()
        return sorted(self.done, key=lambda r: (r.session, r.seq))


def replay(graphs: Sequence, streams: Sequence[Sequence[Tuple[np.ndarray, np.ndarray]]], slots: int = 4,
           rate_hz: Optional[float] = None, seed: int = 0, **launch) -> Dict[str, object]:
    """Serves every session's batch stream.  rate_hz=None: closed loop (each
    session submits its next batch when the previous one completes); else
    open loop with Poisson arrivals at rate_hz over all sessions.  `launch`
    holds ImceState launch settings (waves_per_cu, donate_interval, ...)."""
    srv = Server(graphs, slots=slots, **launch)
    reqs = [Request(s, k, np.asarray(a, np.uint32), np.asarray(b, np.uint32))
            for s, stream in enumerate(streams) for k, (a, b) in enumerate(stream)]
    total = len(reqs)
    t0 = time.perf_counter()
    if rate_hz is None:
        # closed loop: each session issues its next batch the moment the
        # previous one completes, so a latency is one batch's own service time
        # plus any wait for a slot shared with other sessions
        nxt = {}
        for r in reqs:
            nxt.setdefault(r.session, []).append(r)
        for q in nxt.values():
            q.sort(key=lambda r: r.seq)

        def follow(done_req):
            q = nxt[done_req.session]
            if q:
                r = q.pop(0)
                r.arrival = time.perf_counter()
                srv.pending.append(r)

        srv.on_done = follow
        for q in nxt.values():
            r = q.pop(0)
            r.arrival = t0
            srv.submit(r)
        done = srv.serve(total)
    else:
        rng = np.random.default_rng(seed)
        order = sorted(reqs, key=lambda r: (r.seq, r.session))
        gaps = rng.exponential(1.0 / rate_hz, size=len(order))
        arrivals = t0 + np.cumsum(gaps)

        def feeder():
            for r, at in zip(order, arrivals):
                now = time.perf_counter()
                if at > now:
                    time.sleep(at - now)
                r.arrival = float(at)
                srv.submit(r)

        th = threading.Thread(target=feeder, daemon=True)
        th.start()
        done = srv.serve(total)
        th.join()
    wall = time.perf_counter() - t0
    lat = [r.latency_ms for r in done if r.error is None]
    out = {"requests": done, "wall_s": wall, "p50_ms": nearest_rank(lat, 50), "p99_ms": nearest_rank(lat, 99),
           "mean_ms": float(np.mean(lat)) if lat else float("nan"), "errors": [r.error for r in done if r.error],
           "max_in_flight": srv.max_in_flight, "max_overlap_sessions": srv.max_overlap_sessions,
           "throughput_batches_per_s": len(done) / wall if wall > 0 else 0.0}
    srv.close()
    return out


def run_alone(g, stream: Sequence[Tuple[np.ndarray, np.ndarray]], **launch) -> List[dict]:
    """The same batches, one at a time, on a fresh state (reference results)."""
    st = ImceState(g, **launch)
    out = [st.add(a, b) for a, b in stream]
    st.close()
    return out


RESULT_KEYS = ("n_applied", "n_skipped", "n_new", "n_del", "hash_new", "hash_del", "count", "set_hash")
