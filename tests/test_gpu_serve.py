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
    ex = [TreeExecutor(t, capacity=4, mode="graph") for t in trees]
    got = {}

    def keep(q, e):
        got[q.qid] = e.marginals(q.slot)

    budget = sum(e.shared_bytes for e in ex) + 6 * max(e.slot_bytes for e in ex)
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
