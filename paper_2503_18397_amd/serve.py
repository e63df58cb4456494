"""Serving loop: build and query requests of mixed sizes against structures
kept resident in HBM.

Requests arrive over time (``Server.submit``).  A scheduler admits them into
a fixed number of slots, each a worker thread with its own HIP stream, as
slots and memory free up: a build needs its workspace and structure bytes
(``vf_plan``), a query its output bytes, and the sum over running work and
resident structures stays within the HBM budget.  Admission is first-fit in
arrival order, so a large build that does not fit yet does not hold back
smaller requests behind it; a query waits until its structure is built.
Work admitted to different slots overlaps on the device.  Query requests
that wait together are merged: when a query is admitted, up to
``coalesce`` - 1 other ready queries (any structures) join it, and the slot
answers all of them with one combined launch (``vf_query_multi``).  Builds
and queries are the library's (``vf_build``, ``vfilter_build``,
``vf_query_multi``); their results are canonical, so a request gives the
same bytes alone, merged and in any mix.

The scheduling core (``Scheduler``) knows nothing about the GPU: it takes
the footprint of a request and an executor callable, which the tests replace
by a CPU stand-in.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Any, Callable


@dataclass
class Request:
    """One build or query.  ``kind`` is "vfunc", "vfilter" or "query";
    builds carry keys (and values for a VFunc), b, eps and seed; a query
    carries the id of the build it asks and its keys."""
    rid: int
    kind: str
    keys: Any
    values: Any = None
    b: int = 8
    eps: float = 0.0175
    seed: int = 0
    target: int | None = None  # query: rid of the build
    arrival: float = 0.0
    # filled in by the scheduler
    admitted: float = 0.0
    done: float = 0.0
    footprint: int = 0
    resident: int = 0  # bytes that stay after the request (a structure)
    result: Any = None
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class Stats:
    completed: list = field(default_factory=list)
    peak_bytes: int = 0
    start: float = 0.0
    end: float = 0.0

    def summary(self) -> dict:
        import numpy as np
        out = {"makespan_s": round(self.end - self.start, 6), "peak_bytes": self.peak_bytes}
        for kind in ("build", "query"):
            rs = [r for r in self.completed
                  if (r.kind == "query") == (kind == "query") and r.error is None]
            if not rs:
                continue
            lat = np.array([r.latency for r in rs]) * 1e3
            keys = sum(int(r.keys.numel()) for r in rs)
            out[kind] = {"count": len(rs), "p50_ms": round(float(np.percentile(lat, 50)), 4),
                         "p99_ms": round(float(np.percentile(lat, 99)), 4),
                         "keys": keys,
                         "keys_per_s": round(keys / max(self.end - self.start, 1e-9), 1)}
        out["errors"] = sum(r.error is not None for r in self.completed)
        return out


class Scheduler:
    """Slots, memory admission and dependencies; ``execute(slot, request,
    target)`` runs a request on a slot and returns its result (called on the
    slot's worker thread).  ``footprint(request)`` returns (bytes while
    running, bytes that stay resident afterwards).  With ``execute_many``
    and ``coalesce`` > 1, queries admitted together run as one group:
    ``execute_many(slot, requests, targets)`` returns their results in
    order."""

    def __init__(self, slots: int, budget: int, execute: Callable, footprint: Callable,
                 execute_many: Callable | None = None, coalesce: int = 1):
        if slots < 1:
            raise ValueError("at least one slot")
        self.budget = budget
        self.execute = execute
        self.execute_many = execute_many
        self.coalesce = max(1, int(coalesce)) if execute_many is not None else 1
        self.groups = 0  # launches of merged query groups (two or more requests)
        self.footprint = footprint
        self.cv = threading.Condition()
        self.queue: deque = deque()
        self.used = 0
        self.built: dict = {}       # rid of a finished build -> its request
        self.failed: set = set()    # rids of builds that failed
        self.free_slots = list(range(slots))
        self.inbox: list = [deque() for _ in range(slots)]
        self.stats = Stats()
        self.pending = 0
        self.closed = False
        self.workers = [threading.Thread(target=self._work, args=(s,), daemon=True)
                        for s in range(slots)]
        for w in self.workers:
            w.start()

    # -- client side
    def submit(self, req: Request) -> None:
        req.arrival = time.perf_counter()
        run, stay = self.footprint(req)
        req.footprint, req.resident = int(run), int(stay)
        with self.cv:
            if self.stats.start == 0.0:
                self.stats.start = req.arrival
            self.queue.append(req)
            self.pending += 1
            self._dispatch()

    def drain(self, timeout: float | None = None) -> Stats:
        with self.cv:
            end = None if timeout is None else time.perf_counter() + timeout
            while self.pending:
                left = None if end is None else end - time.perf_counter()
                if left is not None and left <= 0:
                    raise TimeoutError(f"{self.pending} requests still pending")
                self.cv.wait(left)
            return self.stats

    def close(self) -> None:
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for w in self.workers:
            w.join()

    def release(self, rid: int) -> None:
        """Drop a resident structure (its bytes become available)."""
        with self.cv:
            req = self.built.pop(rid, None)
            if req is not None:
                self.used -= req.resident
                req.result = None
                self._dispatch()

    # -- scheduling (called with the lock held)
    def _ready(self, req: Request) -> bool | None:
        """True: can run now; False: must wait; None: can never run."""
        if req.kind == "query":
            if req.target in self.failed:
                return None
            if req.target not in self.built:
                return False
        if req.footprint > self.budget:
            return None
        return self.used + req.footprint <= self.budget

    def _dispatch(self) -> None:
        keep = deque()
        while self.queue:
            req = self.queue.popleft()
            if not self.free_slots:
                keep.append(req)
                continue
            ok = self._ready(req)
            if ok is None:
                req.error = "cannot run (too large for the budget, or its build failed)"
                req.done = time.perf_counter()
                if req.kind != "query":
                    self.failed.add(req.rid)  # its queries fail too, not wait
                self._finish(req)
                continue
            if not ok:
                keep.append(req)
                continue
            slot = self.free_slots.pop()
            group = [req]
            if req.kind == "query" and self.coalesce > 1:
                # ready queries behind it (any structure) join its launch
                rest = deque()
                while self.queue:
                    other = self.queue.popleft()
                    if (len(group) < self.coalesce and other.kind == "query"
                            and self._ready(other)
                            and self.used + req.footprint
                            + sum(g.footprint for g in group[1:]) + other.footprint
                            <= self.budget):
                        group.append(other)
                    else:
                        rest.append(other)
                self.queue = rest
            now = time.perf_counter()
            for g in group:
                self.used += g.footprint
                g.admitted = now
            self.stats.peak_bytes = max(self.stats.peak_bytes, self.used)
            if len(group) > 1:
                self.groups += 1
            self.inbox[slot].append(group)
            self.cv.notify_all()
        self.queue = keep

    def _finish(self, req: Request) -> None:
        self.stats.completed.append(req)
        self.stats.end = max(self.stats.end, req.done)
        self.pending -= 1
        self.cv.notify_all()

    # -- slot workers
    def _work(self, slot: int) -> None:
        while True:
            with self.cv:
                while not self.inbox[slot] and not self.closed:
                    self.cv.wait()
                if not self.inbox[slot]:
                    return
                group = self.inbox[slot].popleft()
                targets = [self.built.get(r.target) if r.kind == "query" else None
                           for r in group]
            try:
                if len(group) == 1:
                    group[0].result = self.execute(slot, group[0], targets[0])
                else:
                    for r, res in zip(group, self.execute_many(slot, group, targets)):
                        r.result = res
            except Exception as e:  # reported per request, the server goes on
                for r in group:
                    r.error = f"{type(e).__name__}: {e}"
            done = time.perf_counter()
            with self.cv:
                for req in group:
                    req.done = done
                    # the running footprint is released; a built structure stays
                    self.used -= req.footprint
                    if req.kind != "query":
                        if req.error is None:
                            self.used += req.resident
                            self.stats.peak_bytes = max(self.stats.peak_bytes, self.used)
                            self.built[req.rid] = req
                        else:
                            self.failed.add(req.rid)
                    self._finish(req)
                self.free_slots.append(slot)
                self._dispatch()


class Server:
    """GPU serving loop: ``slots`` worker streams on one device, admission by
    HBM footprint within ``budget`` bytes (structures stay resident); up to
    ``coalesce`` waiting queries share one combined launch."""

    def __init__(self, slots: int = 4, budget: int = 200 << 30, device: str = "cuda:0",
                 coalesce: int = 16):
        import torch

        import paper_2503_18397_amd as vf
        self.vf = vf
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.sched = Scheduler(slots, budget, self._execute, self._footprint,
                               execute_many=self._execute_many,
                               coalesce=min(coalesce, vf.VF_QUERY_MULTI_MAX))

    def _footprint(self, req: Request):
        vf = self.vf
        if req.kind == "query":
            return req.keys.numel() * 8, 0
        sz = vf.vf_plan(req.keys.numel(), req.b, req.eps, req.kind == "vfilter")
        return sz.workspace_bytes + sz.structure_bytes, sz.structure_bytes

    def _execute(self, slot: int, req: Request, target):
        torch, vf = self.torch, self.vf
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            if req.kind == "query":
                st = target.result
                out = st.query(req.keys, stream=stream)
                stream.synchronize()
                return out
            st = vf.Structure.build(req.keys, None if req.kind == "vfilter" else req.values,
                                    b=req.b, eps=req.eps, seed=req.seed, stream=stream)
            stream.synchronize()
            st.release_workspace()
            if st.rc != vf.VF_OK:
                raise vf.VFError(st.rc, "build")
            return st

    def _execute_many(self, slot: int, reqs: list, targets: list) -> list:
        torch, vf = self.torch, self.vf
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            outs = vf.query_many([(t.result, r.keys) for r, t in zip(reqs, targets)],
                                 stream=stream)
            stream.synchronize()
        return outs

    @property
    def merged_launches(self) -> int:
        """Combined launches that answered two or more queries."""
        return self.sched.groups

    def submit(self, req: Request) -> None:
        self.sched.submit(req)

    def drain(self, timeout: float | None = None) -> Stats:
        return self.sched.drain(timeout)

    def close(self) -> None:
        self.sched.close()


def poisson_trace(seed: int, builds: int, queries: int, build_rate: float, query_rate: float,
                  n_lo: int = 1000, n_hi: int = 10_000_000, q_lo: int = 1,
                  q_hi: int = 1_000_000, bits=(4, 8, 16), member_share: float = 0.9):
    """Arrival times and shapes of a mixed request stream: builds and query
    batches arrive as two Poisson processes; build sizes are log-uniform in
    [n_lo, n_hi], b uniform over bits, VFunc and VFilter alternate at random
    1:1; query batches have log-uniform sizes in [q_lo, q_hi], target a build
    that arrived before them and ask member keys with probability
    member_share.  Returns a list of dicts sorted by time."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    tb = np.cumsum(rng.exponential(1.0 / build_rate, builds))
    tq = np.cumsum(rng.exponential(1.0 / query_rate, queries)) + tb[0]
    ev = []
    for i, t in enumerate(tb):
        n = int(np.floor(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        ev.append({"t": float(t), "kind": "vfunc" if rng.random() < 0.5 else "vfilter",
                   "n": n, "b": int(rng.choice(bits)), "id": i})
    for t in tq:
        before = [e["id"] for e in ev[:builds] if e["t"] <= t]
        q = int(np.floor(np.exp(rng.uniform(np.log(q_lo), np.log(q_hi)))))
        ev.append({"t": float(t), "kind": "query", "n": q,
                   "target": int(rng.choice(before)) if before else 0,
                   "members": float(member_share)})
    ev.sort(key=lambda e: e["t"])
    return ev
