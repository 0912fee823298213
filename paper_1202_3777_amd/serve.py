"""Serving loop: evidence queries on many resident junction trees.

Every tree is compiled once and stays on the device with its index maps and
initial tables (Sec. 3.2: the mappings are built when the tree is
established).  Each tree owns a HIP stream and a fixed number of evidence
slots.  Queries arrive over time; the loop

  1. retires finished batches (a device event per batch) and frees their
     slots and memory,
  2. admits waiting queries in arrival order while their HBM footprint (one
     evidence slot of their tree) fits the budget -- queries that arrive while
     others run are admitted as slots and memory free up,
  3. launches, for every tree that is idle and has admitted queries, one
     propagation over those queries packed into slots 0..k-1.

Batches of different trees run concurrently on their own streams, so work
of queries that arrived at different times overlaps on the device.  A
query's result does not depend on the batch it lands in: every slot's
summation order is fixed by its tree alone.

Latency is measured from the arrival time to the device completion time of
the query's batch (device events mapped onto the host clock), so it does
not include the loop's polling delay.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Query:
    qid: int
    tree: int
    ev_vars: np.ndarray
    ev_states: np.ndarray
    arrival: float                      # seconds on the loop clock
    admitted: Optional[float] = None
    launched: Optional[float] = None
    done: Optional[float] = None        # device completion, loop clock
    slot: Optional[int] = None
    batch: Optional[int] = None
    status: str = "pending"             # pending, admitted, running, done, cancelled, rejected
    log_z: Optional[float] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class AdmissionError(RuntimeError):
    pass


class TreeExecutor:
    """One resident tree on the GPU: a JunctionTree with its own stream."""

    def __init__(self, inst, capacity: int, mode: str = "graph", device: str = "cuda:0"):
        import torch
        from . import jt
        self.torch = torch
        self.jt = jt
        self.mode = mode
        self.stream = torch.cuda.Stream(torch.device(device))
        self.tree = jt.JunctionTree(inst.card, inst.clique_off, inst.clique_vars, inst.parent, inst.potentials,
                                    n_slots=capacity, device=device, stream=self.stream)
        self.capacity = capacity
        self.slot_bytes = self.tree.query(jt.JT_Q_SLOT_BYTES)
        self.shared_bytes = self.tree.query(jt.JT_Q_SHARED_BYTES)
        self._event = None

    def launch(self, queries: Sequence[Query]):
        for k, q in enumerate(queries):
            self.tree.set_evidence(k, q.ev_vars, q.ev_states)
        self.tree.propagate(self.mode, n_active=len(queries))
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        self._event = ev
        return ev

    def done(self, ev) -> bool:
        return ev.query()

    def log_z(self, slot: int) -> float:
        return self.jt.jt_marginal(self.tree.handle, slot, 0, None)

    def marginals(self, slot: int):
        return self.tree.marginals_all(slot)


class Clock:
    """Maps device events onto the host loop clock."""

    def __init__(self, torch_mod=None):
        self.torch = torch_mod
        self.t0 = time.perf_counter()
        self.ref = None
        if torch_mod is not None:
            torch_mod.cuda.synchronize()
            self.ref = torch_mod.cuda.Event(enable_timing=True)
            self.ref.record()
            torch_mod.cuda.synchronize()
            self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def event_time(self, ev) -> float:
        if self.ref is None:
            return ev.t_done
        return self.ref.elapsed_time(ev) * 1e-3


class Server:
    def __init__(self, executors: List, budget_bytes: int, clock: Optional[Clock] = None,
                 on_done: Optional[Callable] = None):
        self.ex = executors
        self.on_done = on_done    # called as on_done(query, executor) before the slot is reused
        self.clock = clock or Clock()
        self.shared = sum(e.shared_bytes for e in executors)
        if self.shared > budget_bytes:
            raise AdmissionError("resident trees alone exceed the HBM budget")
        self.budget = budget_bytes
        self.in_use = self.shared
        self.pending: Deque[Query] = collections.deque()
        self.waiting: List[Deque[Query]] = [collections.deque() for _ in executors]
        self.running: List[Optional[tuple]] = [None] * len(executors)
        self.finished: List[Query] = []
        self.n_batches = 0
        self.batch_sizes: List[int] = []

    # -- admission ------------------------------------------------------
    def submit(self, q: Query):
        e = self.ex[q.tree]
        if self.shared + e.slot_bytes > self.budget:
            q.status = "rejected"
            self.finished.append(q)
            raise AdmissionError(f"query {q.qid}: one slot of tree {q.tree} does not fit the budget")
        self.pending.append(q)

    def cancel(self, q: Query) -> bool:
        """Cancel a query that has not started running."""
        if q.status == "pending":
            self.pending.remove(q)
        elif q.status == "admitted":
            self.waiting[q.tree].remove(q)
            self.in_use -= self.ex[q.tree].slot_bytes
        else:
            return False
        q.status = "cancelled"
        self.finished.append(q)
        return True

    def _admit(self, now: float):
        while self.pending:
            q = self.pending[0]
            e = self.ex[q.tree]
            w = self.waiting[q.tree]
            if self.in_use + e.slot_bytes > self.budget or len(w) >= e.capacity:
                break                        # arrival order: the head waits for room
            self.pending.popleft()
            self.in_use += e.slot_bytes
            q.status = "admitted"
            q.admitted = now
            w.append(q)

    # -- batches ----------------------------------------------------------
    def _retire(self):
        for t, r in enumerate(self.running):
            if r is None:
                continue
            ev, batch = r
            if not self.ex[t].done(ev):
                continue
            tdone = self.clock.event_time(ev)
            for q in batch:
                q.done = tdone
                q.status = "done"
                if self.on_done is not None:
                    self.on_done(q, self.ex[t])
                self.finished.append(q)
                self.in_use -= self.ex[t].slot_bytes
            self.running[t] = None

    def _launch(self, now: float):
        for t, w in enumerate(self.waiting):
            if self.running[t] is not None or not w:
                continue
            e = self.ex[t]
            batch = [w.popleft() for _ in range(min(len(w), e.capacity))]
            for k, q in enumerate(batch):
                q.slot = k
                q.batch = self.n_batches
                q.status = "running"
                q.launched = now
            ev = e.launch(batch)
            self.running[t] = (ev, batch)
            self.n_batches += 1
            self.batch_sizes.append(len(batch))

    def step(self):
        now = self.clock.now()
        self._retire()
        self._admit(now)
        self._launch(now)

    def busy(self) -> bool:
        return bool(self.pending) or any(self.waiting) or any(r is not None for r in self.running)

    def run(self, queries: Sequence[Query], idle_sleep: float = 20e-6, max_seconds: float = 120.0):
        """Feed queries at their arrival times and serve until all finish."""
        order = sorted(queries, key=lambda q: q.arrival)
        i = 0
        t_end = self.clock.now() + max_seconds
        while i < len(order) or self.busy():
            now = self.clock.now()
            if now > t_end:
                raise TimeoutError("serving loop exceeded its time limit")
            while i < len(order) and order[i].arrival <= now:
                self.submit(order[i])
                i += 1
            before = self.n_batches
            self.step()
            if self.n_batches == before and (i >= len(order) or order[i].arrival > self.clock.now()):
                time.sleep(idle_sleep)
        return self.finished


def make_queries(trees, n: int, rate: Optional[float], seed: int = 0, obs=(1, 8), t_start: float = 0.0):
    """n queries, uniform tree, uniform observed variables and states.
    rate=None: all arrive at t_start (saturation); else Poisson at `rate`/s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = t_start
    out = []
    for k in range(n):
        if rate is not None:
            t += rng.exponential(1.0 / rate)
        ti = int(rng.integers(0, len(trees)))
        inst = trees[ti]
        m = int(rng.integers(obs[0], obs[1] + 1))
        vs = np.sort(rng.choice(inst.n_vars, size=min(m, inst.n_vars), replace=False)).astype(np.int32)
        st = np.asarray([int(rng.integers(0, int(inst.card[v]))) for v in vs], dtype=np.int32)
        out.append(Query(qid=k, tree=ti, ev_vars=vs, ev_states=st, arrival=t))
    return out


def latency_stats(done: Sequence[Query]) -> Dict[str, float]:
    lat = np.asarray([q.latency for q in done if q.status == "done"], dtype=np.float64)
    if lat.size == 0:
        return {"n": 0}
    span = max(q.done for q in done if q.status == "done") - min(q.arrival for q in done)
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "queries_per_s": float(lat.size / span) if span > 0 else math.inf}
