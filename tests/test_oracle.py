"""Pins of the FP64 oracle against things other than itself.

Each check fixes part of the oracle by what the paper prints or what the
mathematics forces:
  * Fig. 2's printed mapping tables (golden fixture);
  * the literal quadratic state-string scan of Sec. 3.1, and numpy's own
    ravel/unravel routines, for the mapping tables on random cliques;
  * the partition invariant: every list has |phi_X|/|phi_S| members;
  * full-joint enumeration on trees of up to 23 binary variables;
  * variable elimination on the full 62-variable binary tree;
  * calibration invariants: neighbours agree on separator marginals and
    every clique yields the same log Z;
  * the closed form Z = 1 (log Z = 0) for conditional tables without
    evidence, and Z_e = P(e) with evidence;
  * the operation counts of Sec. 3.4;
  * the 0/0 rule and zero-probability evidence;
  * rejection of inputs that are not junction trees.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1202_3777_amd.instances import from_arrays, make_instance
from tests.exact import brute_force, numpy_class_labels, variable_elimination

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_fig2_mapping_tables():
    g = json.load(open(os.path.join(GOLDEN, "fig2_maps.json")))
    # the right clique of Fig. 2 is a child of the root {A, B, D}
    inst = from_arrays(g["card"], [g["X_i"], g["X_k"]], [-1, 0])
    plan = oracle.Plan.from_instance(inst)
    assert list(plan.sep_vars(1)) == g["S"]
    assert plan.mu(1, 1).tolist() == g["mu_X_i"]
    assert plan.mu(1, 0).tolist() == g["mu_X_k"]
    # the literal per-entry scan of Sec. 3.1 gives the same printed lists
    assert oracle.mu_scan_literal(g["card"], g["X_i"], g["S"]).tolist() == g["mu_X_i"]
    assert oracle.mu_scan_literal(g["card"], g["X_k"], g["S"]).tolist() == g["mu_X_k"]


@pytest.mark.parametrize("name,seed", [("c1", 0), ("c1", 1), ("c4", 0), ("c4", 3)])
def test_mapping_tables_three_ways(name, seed):
    inst = make_instance(name, seed)
    plan = oracle.Plan.from_instance(inst)
    checked = 0
    for c in range(inst.n_cliques):
        p = int(inst.parent[c])
        if p < 0:
            continue
        sv = plan.sep_vars(c)
        assert list(sv) == sorted(set(inst.vars_of(c)) & set(inst.vars_of(p)))
        for side, x in ((0, c), (1, p)):
            xv = inst.vars_of(x)
            mu = plan.mu(c, side)
            size = inst.table_size(x)
            ssize = int(np.prod(inst.card[sv], dtype=np.int64))
            # partition invariant
            assert mu.shape == (ssize, size // ssize)
            assert np.array_equal(np.sort(mu.reshape(-1)), np.arange(size))
            # ascending r inside each list
            assert np.all(np.diff(mu, axis=1) > 0)
            # numpy's index routines
            lab = numpy_class_labels(inst.card, xv, sv)
            assert np.array_equal(plan.csm_map(c, side), lab)
            # the literal quadratic scan, on tables small enough for it
            if size * ssize <= 200_000:
                assert np.array_equal(oracle.mu_scan_literal(inst.card, xv, sv), mu)
                checked += 1
    assert checked > 0


def _assert_close(a, b, tol):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    err = np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)
    assert err <= tol, err


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_small_binary_trees(seed):
    k = 3 + seed % 5                    # 3..7 cliques, at most 23 variables
    inst = make_instance("c1", seed, n_cliques=k, n_obs=(0, 3))
    plan = oracle.Plan.from_instance(inst)
    ev, st = inst.evidence[0]
    res = plan.run(inst.potentials, ev, st)
    assert res["status"] == oracle.OK
    z, margs = brute_force(inst, ev, st)
    assert abs(res["logz"] - np.log(z)) <= 1e-12 * max(1.0, abs(np.log(z)))
    for c in range(inst.n_cliques):
        _assert_close(plan.marginal(res, c), margs[c], 1e-12)


def test_bruteforce_other_root():
    # root not at clique 0: a chain 1 <- 0 <- 2 rooted at clique 1
    card = [2, 3, 2, 2, 3]
    cliques = [[0, 1, 2], [1, 2, 3], [2, 0, 4]]
    inst = from_arrays(card, cliques, [1, -1, 0], seed=5, evidence=[([4], [2])])
    plan = oracle.Plan.from_instance(inst)
    res = plan.run(inst.potentials, [4], [2])
    z, margs = brute_force(inst, [4], [2])
    assert abs(res["logz"] - np.log(z)) < 1e-12
    for c in range(3):
        _assert_close(plan.marginal(res, c), margs[c], 1e-12)


def test_two_clique_direct_sum():
    # special case: with two cliques the calibrated separator marginal is the
    # normalized sum of the product table over the non-separator variables
    card = [3, 2, 4]
    inst = from_arrays(card, [[0, 1], [1, 2]], [-1, 0], seed=11)
    plan = oracle.Plan.from_instance(inst)
    res = plan.run(inst.potentials)
    t0 = inst.table(0).astype(np.float64).reshape(3, 2)
    t1 = inst.table(1).astype(np.float64).reshape(2, 4)
    pb = t0.sum(axis=0) * t1.sum(axis=1)
    m1 = plan.marginal(res, 1).reshape(2, 4)
    _assert_close(m1.sum(axis=1), pb / pb.sum(), 1e-14)
    assert abs(res["logz"] - np.log(pb.sum())) < 1e-13


def test_variable_elimination_full_c1():
    inst = make_instance("c1", 0)
    plan = oracle.Plan.from_instance(inst)
    ev, st = inst.evidence[0]
    res = plan.run(inst.potentials, ev, st)
    assert res["status"] == oracle.OK
    for c in range(inst.n_cliques):
        z, m = variable_elimination(inst, ev, st, query=inst.vars_of(c))
        if c == 0:
            assert abs(res["logz"] - np.log(z)) <= 1e-12 * abs(np.log(z))
        _assert_close(plan.marginal(res, c), m, 1e-12)


def _check_invariants(inst, res, plan, tol):
    lz = res["logz_per_clique"]
    assert np.max(np.abs(lz - res["logz"])) <= tol * max(1.0, abs(res["logz"]))
    for c in range(inst.n_cliques):
        m = plan.marginal(res, c)
        assert abs(m.sum() - 1.0) < 1e-12
        p = int(inst.parent[c])
        if p < 0:
            continue
        sv = plan.sep_vars(c)
        ssize = int(np.prod(inst.card[sv], dtype=np.int64))
        a = np.bincount(numpy_class_labels(inst.card, inst.vars_of(c), sv), weights=m, minlength=ssize)
        mp = plan.marginal(res, p)
        b = np.bincount(numpy_class_labels(inst.card, inst.vars_of(p), sv), weights=mp, minlength=ssize)
        _assert_close(a, b, tol)


@pytest.mark.parametrize("name,seed,kw", [
    ("c1", 0, {}), ("c1", 2, {}), ("c4", 0, dict(n_slots=2)), ("c4", 1, dict(n_slots=2)),
    ("c2", 0, dict(n_cliques=5)), ("c3", 0, dict(n_cliques=6)),
])
def test_calibration_invariants(name, seed, kw):
    inst = make_instance(name, seed, **kw)
    plan = oracle.Plan.from_instance(inst)
    for slot in range(inst.n_slots):
        ev, st = inst.evidence[slot]
        res = plan.run(inst.potentials, ev, st)
        assert res["status"] == oracle.OK
        _check_invariants(inst, res, plan, 1e-11)


@pytest.mark.parametrize("name,kw", [("c1", {}), ("c4", {}), ("c2", dict(n_cliques=4))])
def test_conditional_tables_partition_function(name, kw):
    inst = make_instance(name, 7, conditional=True, **kw)
    plan = oracle.Plan.from_instance(inst)
    res = plan.run(inst.potentials)
    # FP32-rounded conditional tables sum to 1 only to ~1e-7 per row
    assert abs(res["logz"]) < 1e-5 * inst.n_cliques
    # with evidence, Z_e is the probability of the evidence
    small = make_instance("c1", 3, conditional=True, n_cliques=6)
    p2 = oracle.Plan.from_instance(small)
    ev, st = small.evidence[0]
    r2 = p2.run(small.potentials, ev, st)
    z, _ = brute_force(small, ev, st)
    z0, _ = brute_force(small)
    assert abs(np.exp(r2["logz"]) - z) < 1e-12
    assert 0.0 < z <= z0 * (1 + 1e-12)


def test_operation_counts_sec34():
    inst = make_instance("c4", 2, n_slots=1)
    plan = oracle.Plan.from_instance(inst)
    ev, st = inst.evidence[0]
    res = plan.run(inst.potentials, ev, st)
    adds = muls = sadds = smuls = 0
    for c in range(inst.n_cliques):
        p = int(inst.parent[c])
        if p < 0:
            continue
        s = plan.sep_size(c)
        xc, xp = inst.table_size(c), inst.table_size(p)
        # collect c -> p and distribute p -> c
        adds += (xc - s) + (xp - s)
        muls += (xp + s) + (xc + s)
        sadds += 2 * (s - 1)
        smuls += 2 * s
    assert res["adds"] == adds
    assert res["muls"] == muls
    assert res["scale_adds"] == sadds
    assert res["scale_muls"] == smuls


def test_zero_over_zero_rule():
    # clique 0 = (A, B), clique 1 = (B, C).  phi_0(., B=1) = 0, so the
    # collect message has a zero entry and the distribute ratio is 0/0 there.
    card = [2, 2, 3]
    t0 = np.array([0.5, 0.0, 0.25, 0.0], dtype=np.float32)
    t1 = np.array([0.2, 0.3, 0.5, 0.1, 0.6, 0.3], dtype=np.float32)
    inst = from_arrays(card, [[0, 1], [1, 2]], [-1, 0], potentials=np.concatenate([t0, t1]))
    plan = oracle.Plan.from_instance(inst)
    for root_first in (False, True):
        if root_first:
            inst = from_arrays(card, [[1, 2], [0, 1]], [-1, 0], potentials=np.concatenate([t1, t0]))
            plan = oracle.Plan.from_instance(inst)
        res = plan.run(inst.potentials, [2], [1])
        assert res["status"] == oracle.OK
        assert np.all(np.isfinite(res["marginals"]))
        z, margs = brute_force(inst, [2], [1])
        for c in range(2):
            _assert_close(plan.marginal(res, c), margs[c], 1e-14)
    # evidence with probability zero
    res = plan.run(inst.potentials, [1], [1])
    assert res["status"] == oracle.ZERO_EVIDENCE
    assert res["logz"] == -np.inf
    assert np.all(res["marginals"] == 0)


@pytest.mark.parametrize("cliques,parent,code", [
    ([[0, 1], [1, 2]], [-1, -1], oracle.E_NOT_JT),            # two roots
    ([[0, 1], [1, 2]], [1, 0], oracle.E_NOT_JT),              # cycle, no root
    ([[0, 1], [1, 2], [2, 0]], [-1, 0, 1], oracle.E_NOT_JT),  # running intersection broken (var 0)
    ([[0, 0], [0, 1]], [-1, 0], oracle.E_ARG),                # duplicate variable
    ([[0, 5], [0, 1]], [-1, 0], oracle.E_ARG),                # variable out of range
    ([[0, 1], [1, 2]], [-1, 7], oracle.E_NOT_JT),             # parent out of range
])
def test_rejects_non_junction_trees(cliques, parent, code):
    card = np.array([2, 2, 2], dtype=np.int32)
    off = np.concatenate([[0], np.cumsum([len(c) for c in cliques])]).astype(np.int64)
    flat = np.array([v for c in cliques for v in c], dtype=np.int32)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.Plan(card, off, flat, np.array(parent, dtype=np.int32))
    assert ei.value.code == code


def test_rejects_bad_evidence():
    inst = make_instance("c1", 0)
    plan = oracle.Plan.from_instance(inst)
    for ev, st in (([0], [2]), ([99], [0]), ([3, 3], [0, 1])):
        with pytest.raises(oracle.OracleError):
            plan.run(inst.potentials, ev, st)
    # a repeated observation with the same state is fine
    assert plan.run(inst.potentials, [3, 3], [1, 1])["status"] == oracle.OK
