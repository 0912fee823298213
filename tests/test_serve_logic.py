"""Serving loop logic on the CPU, with a stand-in executor whose batches
finish after a simulated device time (no GPU): admission by footprint,
arrival order, continuous batching, overlap across trees, cancellation,
rejection and the loop's time limit."""
import time

import numpy as np
import pytest

from paper_1202_3777_amd.serve import AdmissionError, Clock, Query, Server, latency_stats, make_queries


class FakeEvent:
    def __init__(self, t_done):
        self.t_done = t_done


class FakeExecutor:
    def __init__(self, clock, capacity=4, slot_bytes=100, shared_bytes=1000, seconds_per_batch=0.004, never=False):
        self.clock = clock
        self.capacity = capacity
        self.slot_bytes = slot_bytes
        self.shared_bytes = shared_bytes
        self.dt = seconds_per_batch
        self.never = never
        self.launches = []

    def launch(self, queries, lane=0):
        t = self.clock.now()
        self.launches.append((t, [q.qid for q in queries]))
        return FakeEvent(float("inf") if self.never else t + self.dt)

    def done(self, ev):
        return self.clock.now() >= ev.t_done


def _queries(n_trees, n, rate, seed=0):
    class T:
        def __init__(self):
            self.n_vars = 10
            self.card = np.full(10, 3, np.int32)
    return make_queries([T() for _ in range(n_trees)], n, rate, seed=seed)


def test_all_served_in_arrival_order_and_batched():
    clock = Clock()
    ex = [FakeExecutor(clock) for _ in range(3)]
    srv = Server(ex, budget_bytes=10 ** 9, clock=clock)
    qs = _queries(3, 60, rate=4000.0)
    done = srv.run(qs, max_seconds=20)
    assert len(done) == 60 and all(q.status == "done" for q in done)
    assert all(q.latency >= 0 and q.done >= q.launched >= q.arrival for q in done)
    assert max(srv.batch_sizes) <= 4 and max(srv.batch_sizes) > 1       # queries were batched
    for e in ex:   # within a tree, batches launch in arrival order
        ids = [i for _, b in e.launches for i in b]
        arr = [qs[i].arrival for i in ids]
        assert arr == sorted(arr)
    st = latency_stats(done)
    assert st["n"] == 60 and st["p99_ms"] >= st["p50_ms"] > 0


def test_budget_limits_admitted_footprint():
    clock = Clock()
    ex = [FakeExecutor(clock, capacity=4, slot_bytes=100, shared_bytes=0) for _ in range(2)]
    srv = Server(ex, budget_bytes=250, clock=clock)       # room for two slots at a time
    qs = _queries(2, 20, rate=None)
    peak = 0
    orig = srv._admit

    def spy(now):
        nonlocal peak
        orig(now)
        peak = max(peak, srv.in_use)
    srv._admit = spy
    done = srv.run(qs, max_seconds=20)
    assert all(q.status == "done" for q in done)
    assert peak <= 250
    assert max(srv.batch_sizes) <= 2
    assert srv.in_use == 0


def test_trees_overlap_and_late_arrivals_join_next_batch():
    clock = Clock()
    ex = [FakeExecutor(clock, capacity=8, seconds_per_batch=0.05) for _ in range(2)]
    srv = Server(ex, budget_bytes=10 ** 9, clock=clock)
    qs = [Query(0, 0, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.0),
          Query(1, 1, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.0),
          Query(2, 0, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.01),
          Query(3, 0, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.02)]
    srv.run(qs, max_seconds=20)
    (t0a, b0a), (t0b, b0b) = ex[0].launches
    (t1a, b1a), = ex[1].launches
    assert b0a == [0] and b0b == [2, 3]           # late arrivals batched together next
    assert abs(t1a - t0a) < 0.04                  # the other tree ran concurrently
    assert t0b >= t0a + 0.05 - 1e-3


def test_cancel_and_reject():
    clock = Clock()
    ex = [FakeExecutor(clock, capacity=1, slot_bytes=100, shared_bytes=0, seconds_per_batch=0.05)]
    srv = Server(ex, budget_bytes=150, clock=clock)
    qs = _queries(1, 3, rate=None)
    for q in qs:
        srv.submit(q)
    srv.step()                      # q0 runs, q1 pending (no room), q2 pending
    assert qs[0].status == "running" and qs[1].status == "pending"
    assert srv.cancel(qs[2]) and qs[2].status == "cancelled"
    assert not srv.cancel(qs[0])
    big = [FakeExecutor(clock, slot_bytes=10 ** 6, shared_bytes=0)]
    srv2 = Server(big, budget_bytes=1000, clock=clock)
    with pytest.raises(AdmissionError):
        srv2.submit(_queries(1, 1, None)[0])
    with pytest.raises(AdmissionError):
        Server([FakeExecutor(clock, shared_bytes=5000)], budget_bytes=1000, clock=clock)


def test_loop_time_limit():
    clock = Clock()
    ex = [FakeExecutor(clock, never=True)]
    srv = Server(ex, budget_bytes=10 ** 9, clock=clock)
    with pytest.raises(TimeoutError):
        srv.run(_queries(1, 2, None), max_seconds=0.2)


def test_full_tree_queue_does_not_block_other_trees():
    # tree 0 gets a burst larger than its queue; a later query for tree 1 is
    # admitted and launched before tree 0's backlog drains
    clock = Clock()
    ex = [FakeExecutor(clock, capacity=2, slot_bytes=1, shared_bytes=0, seconds_per_batch=0.02) for _ in range(2)]
    srv = Server(ex, budget_bytes=10 ** 9, clock=clock)
    qs = [Query(qid=k, tree=0, ev_vars=np.zeros(0, np.int32), ev_states=np.zeros(0, np.int32), arrival=0.0)
          for k in range(8)]
    qs.append(Query(qid=8, tree=1, ev_vars=np.zeros(0, np.int32), ev_states=np.zeros(0, np.int32), arrival=0.001))
    done = srv.run(qs, max_seconds=20)
    assert all(q.status == "done" for q in done)
    last0 = max(q.launched for q in qs if q.tree == 0)
    assert qs[8].launched < last0


def test_lanes_overlap_batches_of_one_tree():
    clock = Clock()
    e = FakeExecutor(clock, capacity=2, slot_bytes=1, shared_bytes=0, seconds_per_batch=0.05)
    e.n_lanes = 2
    srv = Server([e], budget_bytes=10 ** 9, clock=clock)
    qs = [Query(qid=k, tree=0, ev_vars=np.zeros(0, np.int32), ev_states=np.zeros(0, np.int32), arrival=0.002 * k)
          for k in range(4)]
    peak = 0
    orig = srv._launch

    def spy(now):
        nonlocal peak
        orig(now)
        peak = max(peak, len(srv.running[0]))
    srv._launch = spy
    done = srv.run(qs, max_seconds=20)
    assert all(q.status == "done" for q in done)
    assert peak == 2                                 # two batches of the same tree in flight
    assert {q.lane for q in qs} == {0, 1}
