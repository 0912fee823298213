"""Seeded synthetic junction-tree instances.

This module only draws random inputs: tree shape, variable cardinalities,
clique variable orders, FP32 potential tables and hard evidence.  It holds
none of the message-passing arithmetic, so both the GPU path and the CPU
oracle take their inputs from here without sharing any of the method.

Conventions (Sec. 2.1 and Sec. 3 of the paper):
  * variables are 0..n_vars-1 with cardinality ``card[v]``;
  * clique ``c`` lists its variables in ``clique_vars[clique_off[c]:
    clique_off[c+1]]``; the listed order is the table layout, row-major with
    the last-listed variable fastest (the reading that Fig. 2's maps pin);
  * ``parent[c]`` is the neighbour towards the designated root, -1 at the root
    (clique 0 here);
  * potentials are FP32, all tables concatenated in clique order;
  * evidence is hard: a list of (variable, state) pairs per evidence slot.

Trees are random recursive trees: clique c >= 1 hangs under a uniformly
chosen earlier clique.  A child takes ``s`` variables sampled from its
parent (the separator) plus fresh variables, so the running-intersection
property holds by construction, and its variable order is shuffled so that
separator variables land at every stride.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Instance:
    name: str
    seed: int
    card: np.ndarray          # int32 [n_vars]
    clique_off: np.ndarray    # int64 [n_cliques + 1]
    clique_vars: np.ndarray   # int32 [clique_off[-1]]
    parent: np.ndarray        # int32 [n_cliques]
    potentials: np.ndarray    # float32 [sum of table sizes]
    table_off: np.ndarray     # int64 [n_cliques + 1] offsets into potentials
    evidence: List[Tuple[np.ndarray, np.ndarray]]  # per slot: (vars, states)

    @property
    def n_vars(self) -> int:
        return int(self.card.shape[0])

    @property
    def n_cliques(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_slots(self) -> int:
        return len(self.evidence)

    def vars_of(self, c: int) -> np.ndarray:
        return self.clique_vars[self.clique_off[c]:self.clique_off[c + 1]]

    def table(self, c: int) -> np.ndarray:
        return self.potentials[self.table_off[c]:self.table_off[c + 1]]

    def table_size(self, c: int) -> int:
        return int(self.table_off[c + 1] - self.table_off[c])

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.card, self.clique_off, self.clique_vars, self.parent,
                  self.potentials):
            h.update(np.ascontiguousarray(a).tobytes())
        for ev, st in self.evidence:
            h.update(np.ascontiguousarray(ev).tobytes())
            h.update(np.ascontiguousarray(st).tobytes())
        return h.hexdigest()

    def total_entries(self) -> int:
        return int(self.table_off[-1])


# Workload recipes.  Sizes follow the five synthetic workloads: a tiny
# binary tree, a large-clique tree, a high-cardinality tree, a batched
# many-small-clique tree and a serving mix of trees.
CONFIGS: Dict[str, dict] = {
    # 20 cliques of 5 binary variables, separators of 2 variables.
    "c1": dict(n_cliques=20, clique_size=(5, 5), cards=(2,), sep_size=(2, 2),
               potentials=("uniform", 0.1, 1.0), n_obs=(3, 3), n_slots=1),
    # 64 cliques of 10 variables of cardinality 4 (1,048,576 entries),
    # separators of 4-6 variables, Dirichlet(1) rows over the innermost
    # variable, 8 observed variables.
    "c2": dict(n_cliques=64, clique_size=(10, 10), cards=(4,), sep_size=(4, 6),
               potentials=("dirichlet_last",), n_obs=(8, 8), n_slots=1),
    # 30 cliques of 3-4 variables with cardinality 32 or 64 (up to 16.7M
    # entries), separators of 1-2 variables, Uniform(0,1), 4 observed.
    "c3": dict(n_cliques=30, clique_size=(3, 4), cards=(32, 64), sep_size=(1, 2),
               potentials=("uniform", 0.0, 1.0), n_obs=(4, 4), n_slots=1),
    # 200 cliques of 6-12 variables of cardinality 2-3, separators of 2-5
    # variables, 256 evidence sets each observing 1-16 variables.
    "c4": dict(n_cliques=200, clique_size=(6, 12), cards=(2, 3), sep_size=(2, 5),
               potentials=("uniform", 0.1, 1.0), n_obs=(1, 16), n_slots=256),
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _draw_tree(rng, n_cliques, clique_size, cards, sep_size):
    card: List[int] = []
    cvars: List[List[int]] = []
    parent = np.full(n_cliques, -1, dtype=np.int32)

    def fresh(k):
        out = []
        for _ in range(k):
            card.append(int(rng.choice(cards)))
            out.append(len(card) - 1)
        return out

    size0 = int(rng.integers(clique_size[0], clique_size[1] + 1))
    root = fresh(size0)
    cvars.append([root[i] for i in rng.permutation(size0)])
    for c in range(1, n_cliques):
        p = int(rng.integers(0, c))
        parent[c] = p
        size = int(rng.integers(clique_size[0], clique_size[1] + 1))
        smax = min(sep_size[1], size - 1, len(cvars[p]))
        smin = min(sep_size[0], smax)
        s = int(rng.integers(smin, smax + 1))
        pv = cvars[p]
        sep = [pv[i] for i in sorted(rng.choice(len(pv), size=s, replace=False))]
        vs = sep + fresh(size - s)
        cvars.append([vs[i] for i in rng.permutation(len(vs))])
    return np.asarray(card, dtype=np.int32), cvars, parent


def _pack(cvars):
    off = np.zeros(len(cvars) + 1, dtype=np.int64)
    for i, v in enumerate(cvars):
        off[i + 1] = off[i] + len(v)
    flat = np.asarray([x for v in cvars for x in v], dtype=np.int32)
    return off, flat


def _table_offsets(card, cvars):
    off = np.zeros(len(cvars) + 1, dtype=np.int64)
    for i, v in enumerate(cvars):
        off[i + 1] = off[i] + int(np.prod([int(card[x]) for x in v], dtype=np.int64))
    return off


def _draw_potentials(rng, card, cvars, table_off, spec):
    out = np.empty(int(table_off[-1]), dtype=np.float32)
    for c, v in enumerate(cvars):
        n = int(table_off[c + 1] - table_off[c])
        if spec[0] == "uniform":
            t = rng.uniform(spec[1], spec[2], size=n)
        elif spec[0] == "dirichlet_last":
            k = int(card[v[-1]])
            t = rng.dirichlet(np.ones(k), size=n // k).reshape(-1)
        else:
            raise ValueError(spec)
        out[table_off[c]:table_off[c + 1]] = t.astype(np.float32)
    return out


def conditional_potentials(rng, card, cvars, parent, table_off):
    """Tables that are conditional distributions of each clique's fresh
    variables given its separator (the root: a joint over its variables).

    Each row (one separator configuration) is a Dirichlet(1) draw over the
    fresh-variable configurations; the array built in (separator vars
    ascending, fresh vars) order is transposed into the clique's listed
    order.  With such tables the represented joint is normalized, so the
    evidence-free partition function is exactly 1.
    """
    out = np.empty(int(table_off[-1]), dtype=np.float32)
    for c, v in enumerate(cvars):
        if parent[c] < 0:
            sep = []
        else:
            pset = set(cvars[parent[c]])
            sep = sorted(x for x in v if x in pset)
        rest = [x for x in v if x not in set(sep)]
        order = sep + rest
        ns = int(np.prod([int(card[x]) for x in sep], dtype=np.int64)) if sep else 1
        nr = int(np.prod([int(card[x]) for x in rest], dtype=np.int64))
        m = rng.dirichlet(np.ones(nr), size=ns)
        t = m.reshape([int(card[x]) for x in order])
        perm = [order.index(x) for x in v]
        t = np.transpose(t, perm)
        out[table_off[c]:table_off[c + 1]] = np.ascontiguousarray(t).reshape(-1)
    return out


def draw_evidence(rng, card, n_obs: Tuple[int, int], n_slots: int):
    ev = []
    nv = int(card.shape[0])
    for _ in range(n_slots):
        k = int(rng.integers(n_obs[0], n_obs[1] + 1))
        k = min(k, nv)
        vs = np.sort(rng.choice(nv, size=k, replace=False)).astype(np.int32)
        st = np.asarray([int(rng.integers(0, int(card[x]))) for x in vs], dtype=np.int32)
        ev.append((vs, st))
    return ev


def make_instance(name: str, seed: int = 0, *, n_cliques: Optional[int] = None,
                  n_slots: Optional[int] = None, conditional: bool = False,
                  n_obs: Optional[Tuple[int, int]] = None) -> Instance:
    """Draw the named workload from ``seed``.

    ``n_cliques`` truncates/extends the tree (e.g. a 7-clique binary tree
    small enough for full-joint enumeration), ``n_slots`` sets the number of
    evidence sets, ``conditional`` replaces the potentials by conditional
    tables (partition function 1), ``n_obs`` overrides the evidence count.
    """
    cfg = dict(CONFIGS[name])
    if n_cliques is not None:
        cfg["n_cliques"] = n_cliques
    if n_slots is not None:
        cfg["n_slots"] = n_slots
    if n_obs is not None:
        cfg["n_obs"] = n_obs
    rng = _rng(seed)
    card, cvars, parent = _draw_tree(rng, cfg["n_cliques"], cfg["clique_size"],
                                     cfg["cards"], cfg["sep_size"])
    table_off = _table_offsets(card, cvars)
    if conditional:
        pot = conditional_potentials(rng, card, cvars, parent, table_off)
    else:
        pot = _draw_potentials(rng, card, cvars, table_off, cfg["potentials"])
    ev = draw_evidence(rng, card, cfg["n_obs"], cfg["n_slots"])
    off, flat = _pack(cvars)
    return Instance(name=name, seed=seed, card=card, clique_off=off,
                    clique_vars=flat, parent=parent, potentials=pot,
                    table_off=table_off, evidence=ev)


def from_arrays(card: Sequence[int], cliques: Sequence[Sequence[int]],
                parent: Sequence[int], potentials: Optional[np.ndarray] = None,
                evidence: Optional[List[Tuple[Sequence[int], Sequence[int]]]] = None,
                seed: int = 0, name: str = "custom") -> Instance:
    """Build an Instance from explicit lists (hand-written test cases).
    Missing potentials are drawn Uniform(0.1, 1) from ``seed``."""
    card = np.asarray(card, dtype=np.int32)
    cvars = [list(map(int, c)) for c in cliques]
    table_off = _table_offsets(card, cvars)
    if potentials is None:
        rng = _rng(seed)
        potentials = rng.uniform(0.1, 1.0, size=int(table_off[-1])).astype(np.float32)
    potentials = np.asarray(potentials, dtype=np.float32)
    assert potentials.shape[0] == int(table_off[-1])
    if evidence is None:
        evidence = [(np.zeros(0, np.int32), np.zeros(0, np.int32))]
    ev = [(np.asarray(v, dtype=np.int32), np.asarray(s, dtype=np.int32)) for v, s in evidence]
    off, flat = _pack(cvars)
    return Instance(name=name, seed=seed, card=card, clique_off=off, clique_vars=flat,
                    parent=np.asarray(parent, dtype=np.int32), potentials=potentials,
                    table_off=table_off, evidence=ev)


# ----------------------------------------------------------------------------
# Serving mix: 16 distinct trees whose total table entries are log-uniform
# in [1e3, 5e7], variable cardinalities 2..64.
# ----------------------------------------------------------------------------

def make_serving_trees(seed: int = 0, n_trees: int = 16, lo: float = 1e3,
                       hi: float = 5e7, max_cliques: int = 64) -> List[Instance]:
    rng = _rng(seed)
    trees = []
    for t in range(n_trees):
        target = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        n_cl = int(rng.integers(4, max_cliques + 1))
        per = max(8.0, target / n_cl)
        card: List[int] = []
        cvars: List[List[int]] = []
        parent = np.full(n_cl, -1, dtype=np.int32)

        def fresh_until(base_vars, size_now):
            vs = list(base_vars)
            size = size_now
            while True:
                k = int(rng.integers(2, 65))
                if size * k > 2.0 * per and len(vs) >= 2:
                    break
                card.append(k)
                vs.append(len(card) - 1)
                size *= k
                if size >= per:
                    break
            return vs

        cvars.append(fresh_until([], 1))
        for c in range(1, n_cl):
            p = int(rng.integers(0, c))
            parent[c] = p
            pv = cvars[p]
            s = int(rng.integers(1, min(3, len(pv)) + 1))
            sep = [pv[i] for i in sorted(rng.choice(len(pv), size=s, replace=False))]
            size = int(np.prod([card[x] for x in sep], dtype=np.int64))
            vs = fresh_until(sep, size)
            if len(vs) == len(sep):           # at least one fresh variable
                card.append(2)
                vs.append(len(card) - 1)
            cvars.append([vs[i] for i in rng.permutation(len(vs))])
        card_a = np.asarray(card, dtype=np.int32)
        table_off = _table_offsets(card_a, cvars)
        pot = _draw_potentials(rng, card_a, cvars, table_off, ("uniform", 0.1, 1.0))
        off, flat = _pack(cvars)
        trees.append(Instance(name=f"serve{t}", seed=seed, card=card_a, clique_off=off,
                              clique_vars=flat, parent=parent, potentials=pot,
                              table_off=table_off, evidence=[]))
    return trees


def make_separator_sweep(sep_vars: int, seed: int = 0, n_cliques: int = 40, fresh: int = 4,
                         card: int = 2, n_obs: int = 2) -> Instance:
    """A tree whose separators all have ``sep_vars`` variables of
    cardinality ``card`` (|phi_S| = card**sep_vars) and whose cliques add
    ``fresh`` variables each: the family over which the speedup is plotted
    against the average separator size (the paper's Fig. 6 ordering)."""
    rng = _rng(seed)
    size = sep_vars + fresh
    card_l: List[int] = [card] * size
    cvars: List[List[int]] = [[int(x) for x in rng.permutation(size)]]
    parent = np.full(n_cliques, -1, dtype=np.int32)
    for c in range(1, n_cliques):
        p = int(rng.integers(0, c))
        parent[c] = p
        pv = cvars[p]
        sep = [pv[i] for i in sorted(rng.choice(len(pv), size=sep_vars, replace=False))]
        new = list(range(len(card_l), len(card_l) + fresh))
        card_l.extend([card] * fresh)
        vs = sep + new
        cvars.append([vs[i] for i in rng.permutation(len(vs))])
    card_a = np.asarray(card_l, dtype=np.int32)
    table_off = _table_offsets(card_a, cvars)
    pot = _draw_potentials(rng, card_a, cvars, table_off, ("uniform", 0.1, 1.0))
    ev = draw_evidence(rng, card_a, (n_obs, n_obs), 1)
    off, flat = _pack(cvars)
    return Instance(name=f"sepsweep{sep_vars}", seed=seed, card=card_a, clique_off=off, clique_vars=flat,
                    parent=parent, potentials=pot, table_off=table_off, evidence=ev)


# ----------------------------------------------------------------------------
# Bayesian networks (the front end's input): a random DAG, conditional
# tables, and evidence sets drawn from the network.
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class BayesNet:
    card: np.ndarray          # int32 [n_vars]
    parent_off: np.ndarray    # int64 [n_vars + 1]
    parents: np.ndarray       # int32 [parent_off[-1]]; table layout (parents..., v)
    cpts: np.ndarray          # float32, the conditional tables concatenated in variable order
    cpt_off: np.ndarray       # int64 [n_vars + 1]

    @property
    def n_vars(self) -> int:
        return int(self.card.shape[0])

    def parents_of(self, v: int) -> np.ndarray:
        return self.parents[self.parent_off[v]:self.parent_off[v + 1]]

    def cpt(self, v: int) -> np.ndarray:
        """P(v | parents) shaped (card of each parent..., card[v])."""
        shape = [int(self.card[p]) for p in self.parents_of(v)] + [int(self.card[v])]
        return self.cpts[self.cpt_off[v]:self.cpt_off[v + 1]].reshape(shape)


def make_bn(seed: int = 0, n_vars: int = 16, max_parents: int = 3, cards=(2, 3), window: Optional[int] = None) -> BayesNet:
    """Variable v picks 0..max_parents parents uniformly among the earlier
    variables (within the last `window` of them when given, which keeps the
    triangulated cliques small on long networks); each row of P(v | parents)
    is a Dirichlet(1) draw."""
    rng = _rng(seed)
    card = np.asarray([int(rng.choice(cards)) for _ in range(n_vars)], dtype=np.int32)
    pa: List[List[int]] = []
    for v in range(n_vars):
        lo = 0 if window is None else max(0, v - window)
        pool = list(range(lo, v))
        k = int(rng.integers(0, min(max_parents, len(pool)) + 1)) if pool else 0
        pa.append([int(x) for x in rng.choice(pool, size=k, replace=False)] if k else [])
    parent_off = np.zeros(n_vars + 1, dtype=np.int64)
    for v in range(n_vars):
        parent_off[v + 1] = parent_off[v] + len(pa[v])
    parents = np.asarray([p for ps in pa for p in ps], dtype=np.int32)
    cpt_off = np.zeros(n_vars + 1, dtype=np.int64)
    tabs = []
    for v in range(n_vars):
        rows = int(np.prod([int(card[p]) for p in pa[v]], dtype=np.int64)) if pa[v] else 1
        t = rng.dirichlet(np.ones(int(card[v])), size=rows).reshape(-1)
        tabs.append(t.astype(np.float32))
        cpt_off[v + 1] = cpt_off[v] + t.shape[0]
    return BayesNet(card=card, parent_off=parent_off, parents=parents, cpts=np.concatenate(tabs), cpt_off=cpt_off)


def sample_bn_evidence(bn: BayesNet, n_sets: int, n_obs: Tuple[int, int], seed: int = 0):
    """Evidence sets drawn from the network: one ancestral sample per set
    (variables in index order, every parent precedes its child), of which a
    uniformly chosen subset of n_obs variables is observed."""
    rng = _rng(seed)
    out = []
    for _ in range(n_sets):
        x = np.zeros(bn.n_vars, dtype=np.int64)
        for v in range(bn.n_vars):
            row = bn.cpt(v)[tuple(int(x[p]) for p in bn.parents_of(v))].astype(np.float64)
            x[v] = int(rng.choice(int(bn.card[v]), p=row / row.sum()))
        k = int(rng.integers(n_obs[0], n_obs[1] + 1))
        vs = np.sort(rng.choice(bn.n_vars, size=min(k, bn.n_vars), replace=False)).astype(np.int32)
        out.append((vs, x[vs].astype(np.int32)))
    return out
