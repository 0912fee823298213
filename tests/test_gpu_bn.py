"""Bayesian-network front end on the GPU: a network compiled to a junction
tree, its conditional tables multiplied into the cliques by the device
(Algorithm 4's Initialization), propagated with evidence, against the
network oracle (plain definitions in FP64, no junction tree): every clique
posterior and log P(e) within 1e-5, log P(no evidence) = 0, the expected
counts of an EM E-step, the M-step, and EM's log-likelihood never
decreasing over iterations."""
import numpy as np
import pytest

from oracle import bn_oracle
from paper_1202_3777_amd.instances import make_bn, sample_bn_evidence

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_3777_amd import jt
    return jt, torch


@pytest.mark.parametrize("seed,n,mp,window,slots", [(0, 12, 3, None, 4), (1, 40, 3, None, 3), (2, 90, 3, 8, 2)])
def test_bn_clique_posteriors(seed, n, mp, window, slots):
    jt, torch = _gpu()
    bn = make_bn(seed, n_vars=n, max_parents=mp, window=window)
    ev = sample_bn_evidence(bn, slots, (1, 6), seed=seed + 10)
    t = jt.BayesNetTree(bn, n_slots=slots)
    for s, (v, st) in enumerate(ev):
        t.set_evidence(s, v, st)
    t.propagate("graph")
    worst = 0.0
    for s, (v, st) in enumerate(ev):
        got, lz = t.marginals_all(s)
        _, pe = bn_oracle.marginal(bn, [], v, st)
        assert abs(lz - np.log(pe)) <= TOL * max(1.0, abs(np.log(pe))), (s, lz, np.log(pe))
        for c in range(t.n_cliques):
            ref = bn_oracle.posterior(bn, list(t.clique_vars_of(c)), v, st).reshape(-1)
            a = got[t.table_off[c]:t.table_off[c + 1]].astype(np.float64)
            err = float(np.max(np.abs(a - ref)) / np.max(ref))
            worst = max(worst, err)
            assert err <= TOL, (s, c, err)
    print(f"[bn] n={n} cliques={t.n_cliques} slots={slots} max_rel_err={worst:.3e}")


def test_bn_no_evidence_partition_function():
    # the device product of the conditional tables is a normalized joint:
    # log Z = 0 without evidence (to the FP32 rounding of the tables)
    jt, torch = _gpu()
    for seed in range(3):
        bn = make_bn(seed + 20, n_vars=60, max_parents=3, window=10)
        t = jt.BayesNetTree(bn, n_slots=1)
        t.set_evidence(0, [], [])
        t.propagate("fused")
        _, lz = t.marginals_all(0)
        print(f"[bn] no-evidence log Z = {lz:.3e}")
        assert abs(lz) < 1e-5


def test_bn_expected_counts_and_em():
    jt, torch = _gpu()
    bn = make_bn(7, n_vars=18, max_parents=3)
    ev = sample_bn_evidence(bn, 8, (3, 9), seed=3)
    t = jt.BayesNetTree(bn, n_slots=len(ev))
    for s, (v, st) in enumerate(ev):
        t.set_evidence(s, v, st)
    t.propagate("graph")
    counts = t.expected_counts().cpu().numpy().astype(np.float64)
    ref = bn_oracle.expected_counts(bn, ev)
    for v in range(bn.n_vars):
        a, b = counts[bn.cpt_off[v]:bn.cpt_off[v + 1]], ref[bn.cpt_off[v]:bn.cpt_off[v + 1]]
        assert np.max(np.abs(a - b)) <= TOL * max(1.0, np.max(b)), v
    # M-step against its plain definition, from the same counts
    new = t.m_step(t.expected_counts(), alpha=0.5).cpu().numpy()
    assert np.allclose(new, bn_oracle.m_step(bn, counts, 0.5), rtol=1e-6, atol=1e-7)
    # EM: the log-likelihood of the evidence sets never decreases, and the
    # device's sum of log Z matches the oracle's on the same tables
    prev = None
    cur = bn
    for it in range(4):
        t.propagate("graph")
        ll = sum(t.marginals_all(s)[1] for s in range(len(ev)))
        ref_ll = bn_oracle.log_likelihood(cur, ev)
        print(f"[bn-em] iteration {it}: log-likelihood {ll:.6f} (oracle {ref_ll:.6f})")
        assert abs(ll - ref_ll) <= TOL * max(1.0, abs(ref_ll))
        if prev is not None:
            assert ll >= prev - 1e-4
        prev = ll
        cpts = t.m_step(t.expected_counts(), alpha=0.0)
        t.set_cpts(cpts)
        import dataclasses
        cur = dataclasses.replace(cur, cpts=cpts.cpu().numpy())
