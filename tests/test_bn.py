"""Bayesian-network front end on the CPU: the compiled junction tree's
structure (host C++ through the C ABI) and the pins of the network oracle.

Structure: every clique is maximal, every family (variable and parents) lies
in the clique it is assigned to (the lowest-id one holding it), the cliques
cover the moral graph's edges, the tree has running intersection (the
library validates it when compiling; checked again here), a cycle among the
parents is refused.

Oracle (oracle/bn_oracle.py) pinned against an explicit enumeration of all
joint states written here, closed forms (a root's posterior without evidence
is its table; fully observed evidence gives one-hot expected counts; the
M-step of counts is their row-normalized frequencies) and normalization."""
import itertools

import numpy as np
import pytest

from oracle import bn_oracle
from paper_1202_3777_amd import jt
from paper_1202_3777_amd.instances import make_bn, sample_bn_evidence


def _enumerate(bn, ev_vars=(), ev_states=()):
    """P(x) for every joint state, evidence applied (dict state -> prob)."""
    ev = dict(zip(map(int, ev_vars), map(int, ev_states)))
    out = {}
    for x in itertools.product(*[range(int(k)) for k in bn.card]):
        if any(x[v] != s for v, s in ev.items()):
            continue
        p = 1.0
        for v in range(bn.n_vars):
            p *= float(bn.cpt(v)[tuple(x[int(u)] for u in bn.parents_of(v)) + (x[v],)])
        out[x] = p
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oracle_against_enumeration(seed):
    bn = make_bn(seed, n_vars=9, max_parents=3, cards=(2, 3))
    ev = sample_bn_evidence(bn, 1, (2, 3), seed=seed)[0]
    joint = _enumerate(bn, *ev)
    pe = sum(joint.values())
    _, z = bn_oracle.marginal(bn, [], *ev)
    assert abs(z - pe) <= 1e-12 * max(1.0, pe)
    for v in range(bn.n_vars):
        fam = [int(u) for u in bn.parents_of(v)] + [v]
        ref = np.zeros([int(bn.card[u]) for u in fam])
        for x, p in joint.items():
            ref[tuple(x[u] for u in fam)] += p
        got = bn_oracle.posterior(bn, fam, *ev)
        assert np.allclose(got, ref / pe, rtol=1e-12, atol=1e-15)


def test_oracle_closed_forms():
    # (the tables are FP32 roundings of normalized rows, so these closed forms
    # hold to the FP32 rounding of the inputs, ~1e-7)
    bn = make_bn(4, n_vars=10, max_parents=2)
    roots = [v for v in range(bn.n_vars) if bn.parent_off[v + 1] == bn.parent_off[v]]
    for r in roots:
        assert np.allclose(bn_oracle.posterior(bn, [r]), bn.cpt(r).astype(np.float64), rtol=1e-6)
    # P(e) of a normalized network sums to one over the observed variable's states
    v = 7
    tot = sum(bn_oracle.marginal(bn, [], [v], [s])[1] for s in range(int(bn.card[v])))
    assert abs(tot - 1.0) < 1e-6
    # fully observed evidence: expected counts are one-hot
    x = [0] * bn.n_vars
    ev = (np.arange(bn.n_vars, dtype=np.int32), np.asarray(x, dtype=np.int32))
    counts = bn_oracle.expected_counts(bn, [ev, ev])
    for u in range(bn.n_vars):
        c = counts[bn.cpt_off[u]:bn.cpt_off[u + 1]]
        assert c.sum() == pytest.approx(2.0) and c[0] == pytest.approx(2.0)
    # M-step: row-normalized counts
    m = bn_oracle.m_step(bn, counts, 0.0)
    for u in range(bn.n_vars):
        rows = m[bn.cpt_off[u]:bn.cpt_off[u + 1]].reshape(-1, int(bn.card[u]))
        assert np.allclose(rows.sum(axis=1), 1.0)
        assert rows[0, 0] == pytest.approx(1.0)


def test_clique_product_definition():
    bn = make_bn(5, n_vars=5, max_parents=2)
    cv = [3, 0, 1]   # any order
    assigned = [v for v in range(bn.n_vars) if set([*map(int, bn.parents_of(v)), v]) <= set(cv)]
    got = bn_oracle.clique_initial_table(bn, cv, assigned)
    shape = [int(bn.card[x]) for x in cv]
    for r, st in enumerate(itertools.product(*[range(k) for k in shape])):
        s = dict(zip(cv, st))
        p = np.float32(1.0)
        for v in sorted(assigned):
            p = np.float32(p * bn.cpt(v)[tuple(s[int(u)] for u in bn.parents_of(v)) + (s[v],)])
        assert got[r] == p


def _structure(bn, n_slots=1):
    h, nbytes, nc = jt.jt_compile_bn(bn.card, bn.parent_off, bn.parents, n_slots)
    off, cv, par, fam = jt.jt_bn_structure(h, bn.n_vars, nc)
    jt.jt_free(h)
    return [list(cv[off[c]:off[c + 1]]) for c in range(nc)], par, fam


@pytest.mark.parametrize("seed,n,mp,window", [(0, 12, 3, None), (1, 40, 3, None), (2, 200, 4, 10), (3, 60, 1, None)])
def test_compiled_structure(seed, n, mp, window):
    bn = make_bn(seed, n_vars=n, max_parents=mp, window=window)
    cliques, par, fam = _structure(bn)
    sets = [set(c) for c in cliques]
    for c in cliques:
        assert c == sorted(c)
    for a in range(len(sets)):
        for b in range(len(sets)):
            assert a == b or not sets[a] <= sets[b], "clique not maximal"
    for v in range(bn.n_vars):
        f = set(map(int, bn.parents_of(v))) | {v}
        assert f <= sets[fam[v]]
        assert all(not f <= sets[c] for c in range(fam[v])), "family not in its lowest-id clique"
        for p in bn.parents_of(v):       # moral edges are covered
            assert any({int(p), v} <= s for s in sets)
    # running intersection: the cliques holding a variable form a subtree
    nc = len(cliques)
    assert (par == -1).sum() == 1
    for x in range(bn.n_vars):
        hold = [c for c in range(nc) if x in sets[c]]
        roots = [c for c in hold if par[c] < 0 or par[c] not in hold]
        assert len(roots) == 1, x


def test_cycle_refused():
    card = np.asarray([2, 2, 2], np.int32)
    parent_off = np.asarray([0, 1, 2, 3], np.int64)
    parents = np.asarray([2, 0, 1], np.int32)
    with pytest.raises(jt.JTError) as ei:
        jt.jt_compile_bn(card, parent_off, parents)
    assert ei.value.code == jt.JT_E_NOT_JUNCTION_TREE
