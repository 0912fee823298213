"""Bayesian-network definitions in plain numpy, FP64 -- TEST INFRASTRUCTURE.

Only the test suite may import this module.  Written from the plain
definitions, with no junction tree, separator, mapping table or message:

  * the joint P(x) = prod_v P(x_v | x_pa(v)) (Sec. 2.1) and, with hard
    evidence e, P(e) = sum over the joint restricted to e;
  * posterior of any variable set Q: P(x_Q | e) = sum over the other
    variables of the restricted joint / P(e) -- by brute force on small
    networks, or by variable elimination (sum variables out one at a time
    from the conditional tables, fewest-neighbour order) on larger ones;
  * expected counts over evidence sets: sum_s P(x_v, x_pa(v) | e_s);
  * the EM M-step: each row of counts + alpha normalized over the child;
  * a clique's initial table: the FP32 product, in ascending variable
    order, of the conditional tables assigned to it (Algorithm 4's
    Initialization, the plain definition of what the product kernel writes).
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np


def _factors(bn):
    fs = []
    for v in range(bn.n_vars):
        vs = [int(p) for p in bn.parents_of(v)] + [v]
        fs.append((vs, bn.cpt(v).astype(np.float64)))
    return fs


def _evidence_factors(bn, ev_vars, ev_states):
    fs = []
    for v, s in zip(ev_vars, ev_states):
        t = np.zeros(int(bn.card[v]), dtype=np.float64)
        t[int(s)] = 1.0
        fs.append(([int(v)], t))
    return fs


def _multiply(a, b, card):
    va, ta = a
    vb, tb = b
    vs = sorted(set(va) | set(vb))
    def expand(v_, t_):
        order = np.argsort(v_)
        t_ = np.transpose(t_, order)
        srt = sorted(v_)
        shape = [int(card[x]) if x in srt else 1 for x in vs]
        return t_.reshape(shape)
    return vs, expand(va, ta) * expand(vb, tb)


def _sum_out(f, v):
    vs, t = f
    k = vs.index(v)
    return [x for x in vs if x != v], t.sum(axis=k)


def marginal(bn, query: Sequence[int], ev_vars=(), ev_states=()) -> Tuple[np.ndarray, float]:
    """(P(x_Q, e) laid out with Q in the given order, P(e)) by variable
    elimination over the conditional tables and evidence indicators."""
    card = bn.card
    fs = _factors(bn) + _evidence_factors(bn, ev_vars, ev_states)
    q = [int(x) for x in query]
    rest = [v for v in range(bn.n_vars) if v not in q]
    while rest:
        # eliminate the variable with the fewest distinct neighbours
        def nbrs(v):
            s = set()
            for vs, _ in fs:
                if v in vs:
                    s |= set(vs)
            return len(s)
        v = min(rest, key=lambda x: (nbrs(x), x))
        rest.remove(v)
        inv = [f for f in fs if v in f[0]]
        fs = [f for f in fs if v not in f[0]]
        if not inv:
            continue
        prod = inv[0]
        for f in inv[1:]:
            prod = _multiply(prod, f, card)
        fs.append(_sum_out(prod, v))
    prod = ([], np.ones(()))
    for f in fs:
        prod = _multiply(prod, f, card)
    vs, t = prod
    # bring to the query order (variables never in any factor stay uniform 1)
    for x in q:
        if x not in vs:
            vs, t = _multiply((vs, t), ([x], np.ones(int(card[x]))), card)
    order = [vs.index(x) for x in q]
    t = np.transpose(t, order)
    return t, float(t.sum())


def posterior(bn, query, ev_vars=(), ev_states=()) -> np.ndarray:
    t, z = marginal(bn, query, ev_vars, ev_states)
    return t / z


def expected_counts(bn, evidence) -> np.ndarray:
    """Concatenated like the conditional tables: sum_s P(x_pa, x_v | e_s)."""
    out = np.zeros(int(bn.cpt_off[-1]), dtype=np.float64)
    for ev_vars, ev_states in evidence:
        for v in range(bn.n_vars):
            fam = [int(p) for p in bn.parents_of(v)] + [v]
            out[bn.cpt_off[v]:bn.cpt_off[v + 1]] += posterior(bn, fam, ev_vars, ev_states).reshape(-1)
    return out


def log_likelihood(bn, evidence) -> float:
    return float(sum(np.log(marginal(bn, [], ev, st)[1]) for ev, st in evidence))


def m_step(bn, counts: np.ndarray, alpha: float) -> np.ndarray:
    out = np.empty(int(bn.cpt_off[-1]), dtype=np.float64)
    for v in range(bn.n_vars):
        k = int(bn.card[v])
        c = counts[bn.cpt_off[v]:bn.cpt_off[v + 1]].reshape(-1, k).astype(np.float64) + alpha
        s = c.sum(axis=1, keepdims=True)
        out[bn.cpt_off[v]:bn.cpt_off[v + 1]] = np.where(s > 0, c / np.where(s > 0, s, 1), 1.0 / k).reshape(-1)
    return out


def clique_initial_table(bn, clique_vars: Sequence[int], assigned: Sequence[int]) -> np.ndarray:
    """FP32 product over the clique's entries (its variables laid out in the
    given order, last fastest) of the tables of the assigned variables, in
    ascending variable order."""
    cv = [int(x) for x in clique_vars]
    shape = [int(bn.card[x]) for x in cv]
    n = int(np.prod(shape, dtype=np.int64))
    states = np.unravel_index(np.arange(n), shape)
    pos = {x: k for k, x in enumerate(cv)}
    out = np.ones(n, dtype=np.float32)
    for v in sorted(int(a) for a in assigned):
        fam = [int(p) for p in bn.parents_of(v)] + [v]
        idx = np.ravel_multi_index(tuple(states[pos[x]] for x in fam), [int(bn.card[x]) for x in fam])
        out = (out * bn.cpts[bn.cpt_off[v]:bn.cpt_off[v + 1]][idx]).astype(np.float32)
    return out
