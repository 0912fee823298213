"""Exact inference by other means, used to pin the oracle.

Written straight from the plain definition of the result: with hard
evidence e, f_e(x) = prod_C phi_C(x_C) * prod_(v,s) [x_v = s],
Z_e = sum_x f_e(x), and P(x_C | e) = sum over the other variables of
f_e / Z_e.  Two independent evaluations:

  * ``brute_force``: materialize f_e over all variables (small trees only);
  * ``variable_elimination``: sum variables out one at a time from the
    factor list (min-degree order), never building the joint.

Neither uses the junction-tree structure, separators, mapping tables or
message passing.
"""
from __future__ import annotations

import string
from typing import Dict, List, Sequence, Tuple

import numpy as np


def _factor(inst, c):
    vs = [int(v) for v in inst.vars_of(c)]
    t = inst.table(c).astype(np.float64).reshape([int(inst.card[v]) for v in vs])
    return vs, t


def brute_force(inst, ev_vars: Sequence[int] = (), ev_states: Sequence[int] = ()):
    nv = inst.n_vars
    card = [int(k) for k in inst.card]
    joint = np.ones(card, dtype=np.float64)
    for c in range(inst.n_cliques):
        vs, t = _factor(inst, c)
        order = np.argsort(vs)
        t = np.transpose(t, order)
        bshape = [1] * nv
        for v in sorted(vs):
            bshape[v] = card[v]
        joint = joint * t.reshape(bshape)
    for v, s in zip(ev_vars, ev_states):
        idx = [slice(None)] * nv
        keep = np.zeros(card[v], dtype=np.float64)
        keep[int(s)] = 1.0
        bshape = [1] * nv
        bshape[int(v)] = card[v]
        joint = joint * keep.reshape(bshape)
    z = joint.sum()
    margs = []
    for c in range(inst.n_cliques):
        vs = [int(v) for v in inst.vars_of(c)]
        other = tuple(a for a in range(nv) if a not in vs)
        m = joint.sum(axis=other)              # axes now in ascending var order
        srt = sorted(vs)
        perm = [srt.index(v) for v in vs]
        m = np.transpose(m, perm).reshape(-1)
        margs.append(m / z if z > 0 else m * 0)
    return z, margs


def _einsum_product_sum(factors: List[Tuple[List[int], np.ndarray]], keep: List[int]):
    """Multiply factors and sum out every variable not in ``keep``."""
    allv = sorted({v for vs, _ in factors for v in vs} | set(keep))
    letters = {v: string.ascii_letters[i] for i, v in enumerate(allv)}
    ops = []
    for vs, t in factors:
        ops.append(t)
        ops.append([allv.index(v) for v in vs])
    out_idx = [allv.index(v) for v in keep]
    if len(allv) > 52:
        raise ValueError("too many variables in one elimination step")
    return np.einsum(*ops, out_idx)


def variable_elimination(inst, ev_vars: Sequence[int] = (), ev_states: Sequence[int] = (),
                         query: Sequence[int] = ()) -> Tuple[float, np.ndarray]:
    """Return (Z_e, P(query vars | e)) with the result's axes in the order of
    ``query`` (flattened row-major, last fastest)."""
    card = [int(k) for k in inst.card]
    factors: List[Tuple[List[int], np.ndarray]] = [_factor(inst, c) for c in range(inst.n_cliques)]
    for v, s in zip(ev_vars, ev_states):
        keep = np.zeros(card[int(v)], dtype=np.float64)
        keep[int(s)] = 1.0
        factors.append(([int(v)], keep))
    query = [int(v) for v in query]
    remaining = sorted({v for vs, _ in factors for v in vs} - set(query))
    while remaining:
        # min-degree: the variable whose elimination touches the fewest others
        best, best_deg = None, None
        for v in remaining:
            nb = set()
            for vs, _ in factors:
                if v in vs:
                    nb.update(vs)
            deg = len(nb)
            if best_deg is None or deg < best_deg:
                best, best_deg = v, deg
        v = best
        touch = [f for f in factors if v in f[0]]
        rest = [f for f in factors if v not in f[0]]
        scope = sorted({u for vs, _ in touch for u in vs} - {v})
        newt = _einsum_product_sum(touch, scope)
        factors = rest + [(scope, newt)]
        remaining.remove(v)
    res = _einsum_product_sum(factors, query)
    z = float(res.sum())
    return z, (res / z).reshape(-1) if z > 0 else res.reshape(-1) * 0


def numpy_class_labels(card: Sequence[int], xvars: Sequence[int], svars: Sequence[int]) -> np.ndarray:
    """Separator index of every clique entry, from numpy's own index
    routines: unravel the flat clique index into per-variable states (C
    order = last variable fastest) and ravel the separator variables' states
    (ascending id order) back into a flat separator index."""
    xshape = [int(card[v]) for v in xvars]
    size = int(np.prod(xshape, dtype=np.int64))
    states = np.unravel_index(np.arange(size), xshape)
    if len(svars) == 0:
        return np.zeros(size, dtype=np.int64)
    sstates = [states[list(xvars).index(v)] for v in svars]
    return np.ravel_multi_index(sstates, [int(card[v]) for v in svars])
