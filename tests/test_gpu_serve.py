"""Served queries on the GPU: continuous batching over several resident
trees gives every query the same posterior it gets alone, and matches the
FP64 oracle within 1e-5."""
import numpy as np
import pytest

import oracle
from paper_1202_3777_amd.instances import make_serving_trees

pytestmark = pytest.mark.gpu


def test_served_equals_alone_and_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_3777_amd import jt
    from paper_1202_3777_amd.serve import Clock, Server, TreeExecutor, latency_stats, make_queries
    trees = make_serving_trees(seed=3, n_trees=4, lo=1e3, hi=2e5, max_cliques=12)
    ex = [TreeExecutor(t, capacity=4, mode="graph", lanes=2) for t in trees]
    got = {}

    def keep(q, e):
        got[q.qid] = e.fetch(q)

    budget = sum(e.shared_bytes for e in ex) + 6 * max(e.query_bytes for e in ex)
    srv = Server(ex, budget_bytes=budget, clock=Clock(torch), on_done=keep)
    qs = make_queries(trees, 48, rate=20000.0, seed=5)
    done = srv.run(qs, max_seconds=60)
    st = latency_stats(done)
    print(f"[serve] {st} batches={srv.n_batches} sizes={sorted(set(srv.batch_sizes))}")
    assert st["n"] == 48
    assert max(srv.batch_sizes) > 1                   # some queries shared a batch
    plans = [oracle.Plan.from_instance(t) for t in trees]
    for q in qs[::4]:
        inst = trees[q.tree]
        alone = jt.JunctionTree(inst.card, inst.clique_off, inst.clique_vars, inst.parent, inst.potentials, 1)
        alone.set_evidence(0, q.ev_vars, q.ev_states)
        alone.propagate("graph")
        a, la = alone.marginals_all(0)
        b, lb = got[q.qid]
        assert np.array_equal(a, b) and la == lb, q.qid
        res = plans[q.tree].run(inst.potentials, q.ev_vars, q.ev_states)
        worst = max(float(np.max(np.abs(b[alone.table_off[c]:alone.table_off[c + 1]] - plans[q.tree].marginal(res, c)))
                          / np.max(plans[q.tree].marginal(res, c))) for c in range(inst.n_cliques))
        assert worst <= 1e-5 and abs(lb - res["logz"]) <= 1e-5 * max(1.0, abs(res["logz"]))


def test_served_full_serving_mix():
    # the exact mix the serving benchmark times (16 trees, 6.4e7 entries,
    # cardinalities up to 64, 8 slots per tree): three served queries per
    # tree, each against the oracle, and one per tree against the same query
    # propagated alone
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_3777_amd import jt
    from paper_1202_3777_amd.serve import Clock, Query, Server, TreeExecutor
    trees = make_serving_trees(seed=0)
    ex = [TreeExecutor(t, capacity=8, mode="graph", lanes=2) for t in trees]
    rng = np.random.Generator(np.random.PCG64(11))
    qs = []
    for ti, inst in enumerate(trees):
        for k in range(3):
            m = int(rng.integers(1, 9))
            vs = np.sort(rng.choice(inst.n_vars, size=min(m, inst.n_vars), replace=False)).astype(np.int32)
            st = np.asarray([int(rng.integers(0, int(inst.card[v]))) for v in vs], dtype=np.int32)
            qs.append(Query(qid=len(qs), tree=ti, ev_vars=vs, ev_states=st, arrival=float(rng.uniform(0, 0.02))))
    got = {}

    def keep(q, e):
        got[q.qid] = e.fetch(q)

    srv = Server(ex, budget_bytes=1 << 40, clock=Clock(torch), on_done=keep)
    done = srv.run(qs, max_seconds=120)
    assert sum(q.status == "done" for q in done) == len(qs)
    worst_all = elem_all = 0.0
    for q in qs:
        inst = trees[q.tree]
        plan = oracle.Plan.from_instance(inst)
        res = plan.run(inst.potentials, q.ev_vars, q.ev_states)
        b, lb = got[q.qid]
        if res["status"] != 0:
            continue
        off = ex[q.tree].table_off
        worst = elem = 0.0
        for c in range(inst.n_cliques):
            ref = plan.marginal(res, c)
            a = b[off[c]:off[c + 1]].astype(np.float64)
            mb = np.max(ref)
            worst = max(worst, float(np.max(np.abs(a - ref)) / mb))
            big = ref >= 1e-3 * mb
            elem = max(elem, float(np.max(np.abs(a[big] - ref[big]) / ref[big])))
        print(f"[serve-c5] tree={q.tree} q={q.qid} entries={inst.total_entries()} max_rel_err={worst:.3e} "
              f"elem_rel_err={elem:.3e} dlogZ={abs(lb - res['logz']):.3e}")
        assert worst <= 1e-5 and elem <= 1e-4 and abs(lb - res["logz"]) <= 1e-5 * max(1.0, abs(res["logz"]))
        worst_all, elem_all = max(worst_all, worst), max(elem_all, elem)
        del plan
        if q.qid % 3 == 0:
            alone = jt.JunctionTree(inst.card, inst.clique_off, inst.clique_vars, inst.parent, inst.potentials, 1)
            alone.set_evidence(0, q.ev_vars, q.ev_states)
            alone.propagate("graph")
            a, la = alone.marginals_all(0)
            assert np.array_equal(a, b) and la == lb, q.qid
            del alone
    print(f"[serve-c5] worst max_rel_err={worst_all:.3e} elem_rel_err={elem_all:.3e} over {len(qs)} queries")
