"""Serving loop: evidence queries on many resident junction trees.

Every tree is compiled once and stays on the device with its index maps and
initial tables (Sec. 3.2: the mappings are built when the tree is
established).  Each tree has a few "lanes": a handle with its own workspace,
stream and a fixed number of evidence slots, so that a tree can run several
batches at once.  Queries arrive over time; the loop

  1. retires finished batches (a device event per batch, recorded after the
     batch's posteriors have been read out into per-query device buffers)
     and hands each result to ``on_done``;
  2. admits waiting queries in arrival order while the device memory their
     results need (one packed posterior buffer each, reserved at admission,
     allocated on the lane's stream when the batch launches, held until the
     result is handed over) fits the budget beside the resident trees; a
     query whose tree already has a full queue is skipped for now, so
     queries for other trees do not wait behind it;
  3. launches, for every tree with admitted queries and an idle lane, one
     propagation over up to ``capacity`` of them, packed into slots 0..k-1,
     and one read-out of their posteriors.

Batches of different trees, and of the same tree on different lanes, run
concurrently on their own streams, so work of queries that arrived at
different times overlaps on the device.  A query's result does not depend
on the batch it lands in: every slot's summation order is fixed by its tree
alone, and evidence-free messages shared inside a batch are bit-identical to
computed ones.

Latency is measured from the arrival time to the device completion of the
query's read-out (device events mapped onto the host clock), so it does not
include the loop's polling delay.
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
    done: Optional[float] = None        # device completion of the read-out, loop clock
    slot: Optional[int] = None
    lane: Optional[int] = None
    batch: Optional[int] = None
    status: str = "pending"             # pending, admitted, running, done, cancelled, rejected
    result: Optional[object] = None     # executor-specific: the query's read-out buffers
    log_z: Optional[float] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class AdmissionError(RuntimeError):
    pass


class _Lane:
    def __init__(self, torch, jt, inst, capacity, device):
        self.stream = torch.cuda.Stream(torch.device(device))
        self.tree = jt.JunctionTree(inst.card, inst.clique_off, inst.clique_vars, inst.parent, inst.potentials,
                                    n_slots=capacity, device=device, stream=self.stream)


class TreeExecutor:
    """One resident tree on the GPU: `lanes` handles, each with its own
    stream, workspace and `capacity` evidence slots."""

    def __init__(self, inst, capacity: int, mode: str = "graph", device: str = "cuda:0", lanes: int = 1):
        import torch
        from . import jt
        self.torch = torch
        self.jt = jt
        self.mode = mode
        self.device = device
        self.capacity = capacity
        self.n_lanes = lanes
        self.lanes = [_Lane(torch, jt, inst, capacity, device) for _ in range(lanes)]
        t0 = self.lanes[0].tree
        self.total_entries = int(t0.table_off[-1])
        self.table_off = t0.table_off
        self.n_cliques = t0.n_cliques
        # resident: every lane's whole workspace; per query: its read-out
        self.shared_bytes = sum(int(l.tree.device_bytes) for l in self.lanes)
        self.query_bytes = 4 * self.total_entries + 8

    def warm(self):
        """Capture the graphs of every batch size on every lane."""
        for l in self.lanes:
            for k in range(1, self.capacity + 1):
                l.tree.propagate(self.mode, n_active=k)

    def alloc_result(self, q: Query, lane: Optional[int] = None):
        """Nothing at admission (the budget reserves the bytes): a batch's
        result buffers are allocated when it launches, on its lane's stream."""
        return None

    def launch(self, queries: Sequence[Query], lane: int):
        """Propagate `queries` in slots 0..k-1 of `lane`, read their results
        out (one device read-out for the batch, into one buffer allocated on
        the lane's stream, each query keeping its own part of it), and return
        an event recorded after that."""
        L = self.lanes[lane]
        torch = self.torch
        k = len(queries)
        for i, q in enumerate(queries):
            L.tree.set_evidence(i, q.ev_vars, q.ev_states)
        L.tree.propagate(self.mode, n_active=k)
        bytes_moved = L.tree.query(self.jt.JT_Q_BYTES_LAST)
        n = self.total_entries
        with torch.cuda.stream(L.stream):
            post = torch.empty(k * n, dtype=torch.float32, device=self.device)
            lz = torch.empty(k, dtype=torch.float64, device=self.device)
        self.jt.jt_read_out(L.tree.handle, 0, k, post.data_ptr(), lz.data_ptr())
        for i, q in enumerate(queries):
            q.result = (post[i * n:(i + 1) * n], lz[i:i + 1])
        bytes_moved += 2 * 4 * n * k
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(L.stream)
        return ev, bytes_moved

    def done(self, ev) -> bool:
        return ev.query()

    def fetch(self, q: Query):
        """The query's posteriors (packed, clique order) and log Z on the host;
        raises the library's zero-evidence error when P(e) = 0."""
        post, lz = q.result
        lzh = float(lz.cpu().numpy()[0])
        if math.isinf(lzh) and lzh < 0:
            raise self.jt.JTError(self.jt.JT_E_ZERO_EVIDENCE, "fetch", "evidence has probability zero")
        return post.cpu().numpy(), lzh

    def marginals(self, slot: int, lane: int = 0):
        return self.lanes[lane].tree.marginals_all(slot)


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
        self.on_done = on_done    # on_done(query, executor): called once the query's result is complete
        self.clock = clock or Clock()
        self.shared = sum(e.shared_bytes for e in executors)
        if self.shared > budget_bytes:
            raise AdmissionError("resident trees alone exceed the HBM budget")
        self.budget = budget_bytes
        self.in_use = self.shared
        self.pending: Deque[Query] = collections.deque()
        self.waiting: List[Deque[Query]] = [collections.deque() for _ in executors]
        self.running: List[Dict[int, tuple]] = [dict() for _ in executors]   # lane -> (event, batch)
        self.finished: List[Query] = []
        self.n_batches = 0
        self.batch_sizes: List[int] = []
        self.table_bytes = 0      # FP32 table bytes the launched batches move (executor-reported)

    @staticmethod
    def _qbytes(e) -> int:
        return int(getattr(e, "query_bytes", getattr(e, "slot_bytes", 0)))

    @staticmethod
    def _lanes(e) -> int:
        return int(getattr(e, "n_lanes", 1))

    # -- admission ------------------------------------------------------
    def submit(self, q: Query):
        e = self.ex[q.tree]
        if self.shared + self._qbytes(e) > self.budget:
            q.status = "rejected"
            self.finished.append(q)
            raise AdmissionError(f"query {q.qid}: its result does not fit the budget beside the resident trees")
        self.pending.append(q)

    def cancel(self, q: Query) -> bool:
        """Cancel a query that has not started running."""
        if q.status == "pending":
            self.pending.remove(q)
        elif q.status == "admitted":
            self.waiting[q.tree].remove(q)
            self._release(q)
        else:
            return False
        q.status = "cancelled"
        self.finished.append(q)
        return True

    def _release(self, q: Query):
        self.in_use -= self._qbytes(self.ex[q.tree])
        q.result = None if self.on_done is None else q.result

    def _admit(self, now: float):
        # arrival order; a query whose tree's queue is full is passed over
        # (it keeps its place), one that does not fit the memory budget stops
        # admission so that later, smaller queries cannot starve it
        skipped: List[Query] = []
        while self.pending:
            q = self.pending.popleft()
            e = self.ex[q.tree]
            w = self.waiting[q.tree]
            if len(w) >= e.capacity * self._lanes(e):
                skipped.append(q)
                continue
            if self.in_use + self._qbytes(e) > self.budget:
                self.pending.appendleft(q)
                break
            self.in_use += self._qbytes(e)
            alloc = getattr(e, "alloc_result", None)
            q.result = alloc(q) if alloc is not None else None
            q.status = "admitted"
            q.admitted = now
            w.append(q)
        for q in reversed(skipped):
            self.pending.appendleft(q)

    # -- batches ----------------------------------------------------------
    def _retire(self):
        for t, runs in enumerate(self.running):
            for lane in list(runs):
                ev, batch = runs[lane]
                if not self.ex[t].done(ev):
                    continue
                tdone = self.clock.event_time(ev)
                for q in batch:
                    q.done = tdone
                    q.status = "done"
                    if self.on_done is not None:
                        self.on_done(q, self.ex[t])
                    self.finished.append(q)
                    self._release(q)
                del runs[lane]

    def _launch(self, now: float):
        for t, w in enumerate(self.waiting):
            e = self.ex[t]
            while w and len(self.running[t]) < self._lanes(e):
                lane = next(k for k in range(self._lanes(e)) if k not in self.running[t])
                batch = [w.popleft() for _ in range(min(len(w), e.capacity))]
                for k, q in enumerate(batch):
                    q.slot = k
                    q.lane = lane
                    q.batch = self.n_batches
                    q.status = "running"
                    q.launched = now
                r = e.launch(batch, lane)
                ev, moved = r if isinstance(r, tuple) else (r, 0)
                self.table_bytes += int(moved)
                self.running[t][lane] = (ev, batch)
                self.n_batches += 1
                self.batch_sizes.append(len(batch))

    def step(self):
        now = self.clock.now()
        self._retire()
        self._admit(now)
        self._launch(now)

    def busy(self) -> bool:
        return bool(self.pending) or any(self.waiting) or any(self.running)

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
