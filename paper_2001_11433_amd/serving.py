"""Online IMCE serving: edge-addition (and deletion) batches handled as they arrive.

Each session owns a device-resident incremental state (graph, clique count
and set hash) and a HIP stream of its own.  Requests (session, batch) enter a
pending queue with their arrival time.  The admission loop starts a request
when (a) its session has room for it (one batch at a time, or two in
pipelined mode), (b) a slot is free, and (c) the device memory of all states
(as each state reports it, `imce_device_bytes`) plus what the batches in
flight and this one are expected to add stays within the budget; a request
that fails (c) while others are in flight waits and is counted as refused.
Admitted requests run concurrently on worker threads, each driving its
session's stream, so their kernels overlap on the device: continuous
batching across sessions.

Pipelined mode (Section 5's two steps per batch): a session's worker submits
batch k+1 (its new-clique search) while batch k's subsumed-clique pass is
still running on the state's second stream, then collects batch k
(`imce_submit` / `imce_collect`).

Latency = completion - arrival (queueing included); p50/p99 by nearest rank.
"""

from __future__ import annotations

import math
import queue
import threading
import time
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import ImceState, _torch


@dataclass
class Request:
    session: int
    seq: int
    src: np.ndarray
    dst: np.ndarray
    remove: bool = False
    arrival: float = 0.0
    start: float = 0.0
    end: float = 0.0
    result: Optional[dict] = None
    error: Optional[str] = None
    refused: int = 0  # times the memory check held it back
    reserved: int = 0  # expected device-memory growth booked at admission

    @property
    def latency_ms(self) -> float:
        return (self.end - self.arrival) * 1e3


def nearest_rank(values: Sequence[float], q: float) -> float:
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, int(math.ceil(q / 100.0 * len(v))))
    return float(v[k - 1])


class Server:
    def __init__(self, graphs: Sequence, slots: int = 4, mem_budget: Optional[int] = None, pipeline: bool = False,
                 **launch):
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
        self.pipeline = pipeline
        self.window = 2 if pipeline else 1  # batches of one session admitted at once
        self.lock = threading.Condition()
        self.pending: List[Request] = []
        self.outstanding = [0] * len(graphs)
        self.in_flight = 0
        self.done: List[Request] = []
        self.max_in_flight = 0
        self.max_overlap_sessions = 0
        self.refusals = 0
        self.on_done = None  # called with each finished request, under the lock
        # memory model: the bytes each state holds and what a batch may add
        # to it, both as the library reports them
        self.state_bytes = [st.device_bytes() for st in self.states]
        # each session's estimate for a batch of up to rho_ref edges, refreshed
        # by the thread driving the state after each of its batches (the state
        # is only ever queried by that thread while it serves)
        self.rho_ref = [8192] * len(graphs)
        self.growth = [st.batch_bytes(8192) for st in self.states]
        self.reserved = 0  # expected growth of the admitted requests
        self.max_bytes_seen = sum(self.state_bytes)
        self.queues = [queue.Queue() for _ in graphs]
        self.workers = []
        if pipeline:
            for s in range(len(graphs)):
                t = threading.Thread(target=self._session_worker, args=(s,), daemon=True)
                t.start()
                self.workers.append(t)

    def close(self):
        for q in self.queues:
            q.put(None)
        for t in self.workers:
            t.join()
        for s in self.states:
            s.close()

    def submit(self, req: Request):
        with self.lock:
            req.arrival = time.perf_counter() if req.arrival == 0.0 else req.arrival
            self.pending.append(req)
            self.lock.notify_all()

    def expected_growth(self, req: Request) -> int:
        s = req.session
        if len(req.src) > self.rho_ref[s]:  # a larger batch than the estimate covers: scale it up
            return int(self.growth[s] * len(req.src) / self.rho_ref[s])
        return self.growth[s]

    def _eligible(self) -> Optional[Request]:
        # the oldest pending request whose session has room and no older batch
        # pending (batches of a session run in order),
        # whose expected memory fits the budget (always when nothing runs)
        for i, r in enumerate(self.pending):
            if self.outstanding[r.session] >= self.window:
                continue
            if any(p.session == r.session and p.seq < r.seq for p in self.pending):
                continue
            total = sum(self.state_bytes) + self.reserved + self.expected_growth(r)
            if total > self.mem_budget and self.in_flight > 0:
                r.refused += 1
                self.refusals += 1
                continue
            return self.pending.pop(i)
        return None

    def _finish(self, req: Request, bytes_before: int, bytes_after: int, growth: int):
        with self.lock:
            self.rho_ref[req.session] = max(self.rho_ref[req.session], len(req.src))
            self.growth[req.session] = growth
            self.outstanding[req.session] -= 1
            self.in_flight -= 1
            self.reserved -= req.reserved
            s = req.session
            self.state_bytes[s] = bytes_after
            self.max_bytes_seen = max(self.max_bytes_seen, sum(self.state_bytes))
            self.done.append(req)
            if self.on_done is not None:
                self.on_done(req)
            self.lock.notify_all()

    def _run(self, req: Request):
        # one request start to end (imce_add_edges / imce_remove_edges)
        torch = self.torch
        st = self.states[req.session]
        before = self.state_bytes[req.session]
        try:
            with torch.cuda.stream(self.streams[req.session]):
                req.start = time.perf_counter()
                req.result = st.remove(req.src, req.dst) if req.remove else st.add(req.src, req.dst)
                req.end = time.perf_counter()
        except Exception as e:  # reported per request
            req.error = repr(e)
            req.end = time.perf_counter()
        self._finish(req, before, st.device_bytes(),
                     st.batch_bytes(max(self.rho_ref[req.session], len(req.src))))

    def _session_worker(self, s: int):
        # pipelined: submit the next admitted batch before collecting the
        # previous one, so its search overlaps the previous subsumed pass
        torch = self.torch
        st = self.states[s]
        q = self.queues[s]
        held = None  # submitted, not collected
        before = self.state_bytes[s]

        def collect(r):
            nonlocal before
            try:
                r.result = st.collect()
            except Exception as e:
                r.error = repr(e)
            r.end = time.perf_counter()
            after = st.device_bytes()
            self._finish(r, before, after, st.batch_bytes(max(self.rho_ref[s], len(r.src))))
            before = after

        with torch.cuda.stream(self.streams[s]):
            while True:
                r = q.get()
                if r is None:
                    break
                r.start = time.perf_counter()
                try:
                    st.submit(r.src, r.dst, remove=r.remove)
                except Exception as e:
                    r.error = repr(e)
                    r.end = time.perf_counter()
                    if held is not None:
                        collect(held)
                        held = None
                    self._finish(r, before, st.device_bytes(),
                                 st.batch_bytes(max(self.rho_ref[s], len(r.src))))
                    continue
                if held is not None:
                    collect(held)
                held = r
                if q.empty():
                    collect(held)
                    held = None
            if held is not None:
                collect(held)

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
                    r.reserved = self.expected_growth(r)
                    self.reserved += r.reserved
                    self.outstanding[r.session] += 1
                    self.in_flight += 1
                    self.max_in_flight = max(self.max_in_flight, self.in_flight)
                    self.max_overlap_sessions = max(self.max_overlap_sessions,
                                                    sum(1 for o in self.outstanding if o > 0))
                    if self.pipeline:
                        self.queues[r.session].put(r)
                    else:
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
           rate_hz: Optional[float] = None, seed: int = 0, pipeline: bool = False, mem_budget: Optional[int] = None,
           removes: Optional[Sequence[Sequence[bool]]] = None, **launch) -> Dict[str, object]:
    """Serves every session's batch stream.  rate_hz=None: closed loop (each
    session keeps one batch outstanding, two when pipelined: the next batch
    arrives when one completes); else open loop with Poisson arrivals at
    rate_hz over all sessions.  `removes[s][k]` marks batch k of session s as
    a deletion.  `launch` holds ImceState launch settings."""
    srv = Server(graphs, slots=slots, mem_budget=mem_budget, pipeline=pipeline, **launch)
    reqs = [Request(s, k, np.asarray(a, np.uint32), np.asarray(b, np.uint32),
                    remove=bool(removes[s][k]) if removes is not None else False)
            for s, stream in enumerate(streams) for k, (a, b) in enumerate(stream)]
    total = len(reqs)
    t0 = time.perf_counter()
    if rate_hz is None:
        # closed loop: each session issues its next batch the moment one of
        # its outstanding batches completes
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
            for _ in range(srv.window):
                if q:
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
           "throughput_batches_per_s": len(done) / wall if wall > 0 else 0.0,
           "refusals": srv.refusals, "refused_requests": sum(1 for r in done if r.refused),
           "max_device_bytes": srv.max_bytes_seen, "mem_budget": srv.mem_budget}
    srv.close()
    return out


def run_alone(g, stream: Sequence[Tuple[np.ndarray, np.ndarray]], removes: Optional[Sequence[bool]] = None,
              **launch) -> List[dict]:
    """The same batches, one at a time, on a fresh state (reference results)."""
    st = ImceState(g, **launch)
    out = [st.remove(a, b) if (removes is not None and removes[k]) else st.add(a, b)
           for k, (a, b) in enumerate(stream)]
    st.close()
    return out


RESULT_KEYS = ("n_applied", "n_skipped", "n_new", "n_del", "hash_new", "hash_del", "count", "set_hash")
