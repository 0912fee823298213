"""Host-side checks of the C-ABI library (no GPU needed).

  * the library loads and exports every function include/jt.h declares;
  * the precomputed cluster-separator mappings are bit-exact against the
    oracle's state-string scan (CSM single table and the paper's mu lists),
    and reproduce Fig. 2;
  * invalid trees, evidence and call orders return the documented status;
  * schedule facts (entries per sweep, algorithmic bytes, launch counts).
"""
import json
import os
import re

import numpy as np
import pytest

import oracle
from paper_1202_3777_amd import jt
from paper_1202_3777_amd.instances import from_arrays, make_instance

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "jt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(jt_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = jt.load()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(jt.EXPORTED) == names


def test_fig2_maps_from_library():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "fig2_maps.json")))
    inst = from_arrays(g["card"], [g["X_i"], g["X_k"]], [-1, 0])
    plan = jt.JunctionTreePlan.from_instance(inst)
    assert plan.mu_lists(1, 1).tolist() == g["mu_X_i"]
    assert plan.mu_lists(1, 0).tolist() == g["mu_X_k"]


@pytest.mark.parametrize("name,seed,kw", [
    ("c1", 0, {}), ("c1", 1, {}), ("c4", 0, {}), ("c4", 2, {}),
    ("c2", 0, dict(n_cliques=6)), ("c3", 0, dict(n_cliques=6)), ("c3", 1, dict(n_cliques=5)),
])
def test_index_maps_bit_exact(name, seed, kw):
    inst = make_instance(name, seed, **kw)
    plan = jt.JunctionTreePlan.from_instance(inst)
    ref = oracle.Plan.from_instance(inst)
    for c in range(inst.n_cliques):
        if inst.parent[c] < 0:
            continue
        assert plan.query(jt.JT_Q_SEP_SIZE, c) == ref.sep_size(c)
        for side in (0, 1):
            assert np.array_equal(plan.index_map(c, side), ref.csm_map(c, side))
            assert np.array_equal(plan.mu_lists(c, side), ref.mu(c, side))


def test_index_maps_odd_shapes():
    # prime cardinality above the tile limit (tile of one entry), a variable
    # of cardinality 1, and a clique joined by an empty separator
    card = [257, 2, 1, 3, 5, 7]
    cliques = [[0, 1], [1, 2, 3], [3, 4, 5], [5]]
    parent = [-1, 0, 1, 2]
    inst = from_arrays(card, cliques, parent)
    plan = jt.JunctionTreePlan.from_instance(inst)
    ref = oracle.Plan.from_instance(inst)
    for c in (1, 2, 3):
        for side in (0, 1):
            assert np.array_equal(plan.index_map(c, side), ref.csm_map(c, side))
    inst2 = from_arrays([2, 3, 4], [[0, 1], [2]], [-1, 0])   # empty separator
    p2 = jt.JunctionTreePlan.from_instance(inst2)
    assert p2.query(jt.JT_Q_SEP_SIZE, 1) == 1
    assert np.array_equal(p2.index_map(1, 1), np.zeros(6, np.int32))


def _compile(card, cliques, parent, n_slots=1):
    off = np.concatenate([[0], np.cumsum([len(c) for c in cliques])]).astype(np.int64)
    flat = np.array([v for c in cliques for v in c], dtype=np.int32)
    return jt.jt_compile_index_maps(np.array(card, np.int32), off, flat, np.array(parent, np.int32), n_slots)


@pytest.mark.parametrize("card,cliques,parent,n_slots,code", [
    ([2, 2, 2], [[0, 1], [1, 2]], [-1, -1], 1, jt.JT_E_NOT_JUNCTION_TREE),          # two roots
    ([2, 2, 2], [[0, 1], [1, 2]], [1, 0], 1, jt.JT_E_NOT_JUNCTION_TREE),            # cycle
    ([2, 2, 2], [[0, 1], [1, 2], [2, 0]], [-1, 0, 1], 1, jt.JT_E_NOT_JUNCTION_TREE),  # running intersection
    ([2, 2, 2], [[0, 0], [0, 1]], [-1, 0], 1, jt.JT_E_ARG),                         # repeated variable
    ([2, 2, 2], [[0, 5], [0, 1]], [-1, 0], 1, jt.JT_E_ARG),                         # variable out of range
    ([2, 0, 2], [[0, 1], [1, 2]], [-1, 0], 1, jt.JT_E_ARG),                         # cardinality 0
    ([2, 2, 2], [[0, 1], [1, 2]], [-1, 9], 1, jt.JT_E_NOT_JUNCTION_TREE),           # parent out of range
    ([2, 2, 2], [[0, 1], [1, 2]], [-1, 0], 0, jt.JT_E_ARG),                         # no slots
    ([3000, 3000, 3000], [[0, 1, 2]], [-1], 1, jt.JT_E_TOO_LARGE),                  # 2.7e10 entries
])
def test_compile_errors(card, cliques, parent, n_slots, code):
    with pytest.raises(jt.JTError) as ei:
        _compile(card, cliques, parent, n_slots)
    assert ei.value.code == code
    assert jt.jt_last_error() != ""


def test_call_order_and_argument_errors():
    inst = make_instance("c1", 0)
    plan = jt.JunctionTreePlan.from_instance(inst)
    h = plan.handle
    with pytest.raises(jt.JTError) as ei:
        jt.jt_propagate(h, jt.JT_MODE_FUSED)          # not bound
    assert ei.value.code == jt.JT_E_STATE
    with pytest.raises(jt.JTError) as ei:
        jt.jt_marginal(h, 0, 0, None)                 # nothing propagated
    assert ei.value.code == jt.JT_E_STATE
    with pytest.raises(jt.JTError) as ei:
        jt.jt_bind(h, 0, plan.device_bytes, 0, 0)     # NULL workspace
    assert ei.value.code == jt.JT_E_ARG
    with pytest.raises(jt.JTError) as ei:
        jt.jt_bind(h, 4096, 16, 8192, 0)              # workspace too small (checked before any copy)
    assert ei.value.code == jt.JT_E_NO_MEM
    with pytest.raises(jt.JTError) as ei:
        jt.jt_bind(h, 4100, plan.device_bytes, 8192, 0)   # misaligned
    assert ei.value.code == jt.JT_E_ARG
    for slot, vs, st in ((1, [0], [0]), (0, [999], [0]), (0, [0], [2]), (0, [3, 3], [0, 1]), (-1, [], [])):
        with pytest.raises(jt.JTError) as ei:
            jt.jt_set_evidence(h, slot, vs, st)
        assert ei.value.code == jt.JT_E_ARG
    jt.jt_set_evidence(h, 0, [3, 3], [1, 1])          # repeated, same state: fine
    with pytest.raises(jt.JTError) as ei:
        jt.jt_get_index_map(h, int(np.where(inst.parent < 0)[0][0]), 0, 32)   # the root has no separator
    assert ei.value.code == jt.JT_E_ARG
    with pytest.raises(jt.JTError):
        jt.jt_query(h, 99)


def _orient(parent, root):
    """Parents of the same tree hung from `root`, and each clique's eccentricity."""
    n = len(parent)
    adj = [[] for _ in range(n)]
    for c in range(n):
        if parent[c] >= 0:
            adj[c].append(int(parent[c]))
            adj[int(parent[c])].append(c)

    def bfs(s):
        d, par, q = [-1] * n, [-1] * n, [s]
        d[s] = 0
        for x in q:
            for y in adj[x]:
                if d[y] < 0:
                    d[y], par[y] = d[x] + 1, x
                    q.append(y)
        return d, par

    ecc = [max(bfs(s)[0]) for s in range(n)]
    return np.array(bfs(root)[1]), ecc


def test_chained_prepasses():
    # a hub with 14 children finishing at heights 0..6 (it is the tree's
    # center, at height 7): its earliest children are absorbed in three
    # chained pre-passes (levels 2, 4, 5; four, four and two messages), each
    # a read and a write of the hub's table more than one pass would make
    from shapes import hub_with_chains
    inst, hub = hub_with_chains(0, n_slots=1)
    plan = jt.JunctionTreePlan.from_instance(inst)
    assert plan.query(jt.JT_Q_ROOT) == hub
    sparent, _ = _orient(inst.parent, hub)
    sizes = np.diff(inst.table_off)
    kids = [np.count_nonzero(sparent == c) for c in range(inst.n_cliques)]
    assert kids[hub] == 14
    base = 0
    for c in range(inst.n_cliques):
        b = 4 * int(sizes[c])
        base += b + (b if kids[c] else 0)
        base += 2 * b if kids[c] == 0 else (kids[c] + 1) * b
    assert plan.query(jt.JT_Q_BYTES_FUSED) == base + 3 * 2 * 4 * int(sizes[hub])


def test_launch_blocks():
    # blocks per launch (per evidence set); on the large-clique tree the level
    # whose work floor pushed it to 1,420 blocks against the default target
    # of 1,280 (one round of resident blocks) is cut into larger blocks that
    # fit one round, while launches only a few blocks over keep theirs
    inst = make_instance("c2", 0)
    plan = jt.JunctionTreePlan.from_instance(inst)
    n = plan.query(jt.JT_Q_N_LAUNCHES_FUSED)
    blocks = [plan.query(jt.JT_Q_FUSED_LAUNCH_BLOCKS, i) for i in range(n)]
    assert all(b >= 1 for b in blocks)
    assert not any(b > 1.02 * 1280 and b < 2 * 1280 for b in blocks), blocks
    with pytest.raises(jt.JTError):
        plan.query(jt.JT_Q_FUSED_LAUNCH_BLOCKS, n)


def _depth(parent, c):
    d = 0
    while parent[c] >= 0:
        c, d = parent[c], d + 1
    return d


@pytest.mark.parametrize("name,kw", [("c1", {}), ("c4", dict(n_slots=1)), ("c2", dict(n_cliques=9)), ("c2", {}),
                                     ("c3", {})])
def test_schedule_facts(name, kw):
    inst = make_instance(name, 1, **kw)
    plan = jt.JunctionTreePlan.from_instance(inst)
    sizes = np.diff(inst.table_off)
    eps = sum(int(sizes[c] + sizes[inst.parent[c]]) for c in range(inst.n_cliques) if inst.parent[c] >= 0)
    assert plan.query(jt.JT_Q_ENTRIES_PER_SWEEP) == eps
    assert plan.query(jt.JT_Q_TOTAL_ENTRIES) == int(sizes.sum())
    # the schedules collect to a center of the tree: its eccentricity is the
    # radius, and the sweeps have radius + 1 levels each
    root = plan.query(jt.JT_Q_ROOT)
    sparent, ecc = _orient(inst.parent, root)
    assert ecc[root] == min(ecc)
    assert plan.query(jt.JT_Q_HEIGHT) == ecc[root] + 1 == plan.query(jt.JT_Q_DEPTH)
    # fused schedule bytes: every clique read once in collect (plus a write of
    # the absorbed table when it has children); in distribute a leaf reads its
    # initial table and writes its posterior, a clique with k children reads
    # its absorbed table k times and writes its posterior once (children in
    # the schedule's orientation)
    # a clique with more than four children and at most 2^22 entries absorbs
    # its earliest-finished children's messages four at a time in pre-passes
    # at earlier collect levels (each after its children's level and the
    # previous pre-pass, before the clique's own level): one more read and
    # write of its table each
    kids = [np.count_nonzero(sparent == c) for c in range(inst.n_cliques)]
    height = [0] * inst.n_cliques
    order = sorted(range(inst.n_cliques), key=lambda c: -_depth(sparent, c))
    for c in order:
        if sparent[c] >= 0:
            height[sparent[c]] = max(height[sparent[c]], height[c] + 1)
    exp = 0
    for c in range(inst.n_cliques):
        b = 4 * int(sizes[c])
        exp += b + (b if kids[c] else 0)
        exp += 2 * b if kids[c] == 0 else (kids[c] + 1) * b
        if kids[c] > 4 and sizes[c] <= 1 << 22:
            hs = sorted(height[x] for x in range(inst.n_cliques) if sparent[x] == c)
            prev, n_pre = -1, kids[c] - 4
            for k0 in range(0, n_pre, 4):
                level = max(prev + 1, hs[min(n_pre, k0 + 4) - 1] + 1)
                if level >= height[c]:
                    break
                exp += 2 * b
                prev = level
    assert plan.query(jt.JT_Q_BYTES_FUSED) == exp
    # one-at-a-time: reset copy, marginalize + in-place scatter per message,
    # total + in-place normalize per clique
    exp_p = sum(8 * int(s) for s in sizes)
    for c in range(inst.n_cliques):
        p = inst.parent[c]
        if p >= 0:
            exp_p += 4 * int(sizes[c]) + 8 * int(sizes[p]) + 4 * int(sizes[p]) + 8 * int(sizes[c])
    exp_p += sum(12 * int(s) for s in sizes)
    assert plan.query(jt.JT_Q_BYTES_PLAIN) == exp_p
    n = inst.n_cliques
    # set-up kernel + reset pass, (marginalize-and-finalize, scatter) per
    # message, totals-and-finalize + normalize at the end
    assert plan.query(jt.JT_Q_N_LAUNCHES_PLAIN) == 2 + 2 * 2 * (n - 1) + 2
    # one pass launch per collect level and per distribute level of every
    # lane; a lane is a set of whole subtrees of the root, and the root's two
    # passes run on the bound stream
    n_lanes = plan.query(jt.JT_Q_N_LANES)
    nlaunch = plan.query(jt.JT_Q_N_LAUNCHES_FUSED)
    # the launches' bytes add up to the propagation's; every launch is a pass
    assert sum(plan.query(jt.JT_Q_FUSED_LAUNCH_BYTES, i) for i in range(nlaunch)) == exp
    assert all(plan.query(jt.JT_Q_FUSED_LAUNCH_KIND, i) == 1 for i in range(nlaunch))
    if n_lanes == 0:
        assert nlaunch == plan.query(jt.JT_Q_HEIGHT) + plan.query(jt.JT_Q_DEPTH)
        return
    n = inst.n_cliques
    lane = [plan.query(jt.JT_Q_CLIQUE_LANE, c) for c in range(n)]
    assert lane[root] == -1 and all(lane[c] == lane[sparent[c]] for c in range(n) if sparent[c] not in (-1, root))
    assert sorted(set(lane) - {-1}) == list(range(n_lanes))
    height = [0] * n
    depth = [0 if c == root else None for c in range(n)]
    order = [root]
    for x in order:
        for c in range(n):
            if sparent[c] == x:
                depth[c] = depth[x] + 1
                order.append(c)
    for c in reversed(order):
        if sparent[c] >= 0:
            height[sparent[c]] = max(height[sparent[c]], height[c] + 1)
    launch_lanes = [plan.query(jt.JT_Q_FUSED_LAUNCH_LANE, i) for i in range(nlaunch)]
    assert launch_lanes.count(-1) == 2
    for l in range(n_lanes):
        members = [c for c in range(n) if lane[c] == l]
        assert launch_lanes.count(l) == len({height[c] for c in members}) + len({depth[c] for c in members})


def test_tuning_changes_cuts_not_work():
    # every shape choice streams the same tables: same entries, same bytes,
    # its own grouping; bad values are refused
    inst = make_instance("c2", 2, n_cliques=12)
    base = jt.JunctionTreePlan.from_instance(inst)
    for tuning in ({"group_min": 4096}, {"group_max": 65536, "group_div": 256}, {"target_blocks": 300},
                   {"max_lanes": 1}, {"task_min": 1}, {"task_min": 1, "target_blocks": 20480}):
        p = jt.JunctionTreePlan.from_instance(inst, tuning=tuning)
        for q in (jt.JT_Q_BYTES_FUSED, jt.JT_Q_BYTES_PLAIN, jt.JT_Q_ENTRIES_PER_SWEEP, jt.JT_Q_ROOT):
            assert p.query(q) == base.query(q)
        if tuning.get("max_lanes") == 1:
            assert p.query(jt.JT_Q_N_LANES) == 0
            assert p.query(jt.JT_Q_N_LAUNCHES_FUSED) == p.query(jt.JT_Q_HEIGHT) + p.query(jt.JT_Q_DEPTH)
    # lanes are disabled: asking for more than one is refused
    for bad in ({"group_min": -1}, {"max_lanes": 9}, {"max_lanes": 2}, {"group_min": 65536, "group_max": 1024},
                {"task_min": -1}):
        with pytest.raises(jt.JTError) as ei:
            jt.JunctionTreePlan.from_instance(inst, tuning=bad)
        assert ei.value.code == jt.JT_E_ARG
    with pytest.raises(ValueError):
        jt.JunctionTreePlan.from_instance(inst, tuning={"tile": 4})


def test_autotuner_picks_the_fastest():
    from paper_1202_3777_amd import tune
    times = {(): 3.0, (("group_min", 4096),): 2.0, (("target_blocks", 1024),): 2.0}
    cands = [{}, {"group_min": 4096}, {"target_blocks": 1024}]
    best, table = tune.choose(cands, lambda c: times[tuple(sorted(c.items()))])
    assert best == {"group_min": 4096}          # the earliest of the two fastest
    assert [t for _, t in table] == [3.0, 2.0, 2.0]
    # a leading candidate timed slow once is timed again before the choice
    seq = {(): [3.0, 3.0, 3.0, 3.0], (("group_min", 4096),): [2.0, 2.0, 2.0, 2.0],
           (("target_blocks", 1024),): [2.5, 1.5, 1.6, 1.5]}
    calls = []

    def timer(c):
        k = tuple(sorted(c.items()))
        calls.append(k)
        return seq[k][sum(1 for x in calls if x == k) - 1]
    best, table = tune.choose(cands, timer, finalists=2, rounds=3)
    assert best == {"target_blocks": 1024}
    assert [t for _, t in table] == [3.0, 2.0, 1.5]
    assert len(calls) == 3 + 2 * 3              # every candidate once, the two leaders thrice more
    for c in tune.DEFAULT_CANDIDATES:            # every default candidate compiles
        jt.JunctionTreePlan.from_instance(make_instance("c1", 0), tuning=c)


def test_merged_compile_structure():
    # merging small separators: fewer compiled cliques, the caller's cliques
    # stay the interface, bounds below 1 are refused
    inst = make_instance("c1", 0)
    h, nbytes, nm = jt.jt_compile_merged(inst.card, inst.clique_off, inst.clique_vars, inst.parent, 4, 4096)
    assert 1 <= nm < inst.n_cliques
    assert jt.jt_query(h, jt.JT_Q_N_COMPILED_CLIQUES) == nm
    assert jt.jt_query(h, jt.JT_Q_TOTAL_ENTRIES) == inst.total_entries()
    for c in range(inst.n_cliques):
        assert jt.jt_query(h, jt.JT_Q_TABLE_SIZE, c) == inst.table_size(c)
    assert all(jt.jt_query(h, jt.JT_Q_COMPILED_TABLE_SIZE, k) <= 4096 for k in range(nm))
    jt.jt_free(h)
    # nothing below the separator bound: the same number of cliques
    h2, _, nm2 = jt.jt_compile_merged(inst.card, inst.clique_off, inst.clique_vars, inst.parent, 1, 1 << 20)
    assert nm2 == inst.n_cliques
    jt.jt_free(h2)
    with pytest.raises(jt.JTError) as ei:
        jt.jt_compile_merged(inst.card, inst.clique_off, inst.clique_vars, inst.parent, 0, 100)
    assert ei.value.code == jt.JT_E_ARG
    # a tree that is not a junction tree is refused before merging
    bad = np.asarray([-1, -1] + list(inst.parent[2:]), np.int32)
    with pytest.raises(jt.JTError) as ei:
        jt.jt_compile_merged(inst.card, inst.clique_off, inst.clique_vars, bad, 4, 4096)
    assert ei.value.code == jt.JT_E_NOT_JUNCTION_TREE


def test_algorithmic_bytes():
    # the fused schedule's algorithmic bytes: per clique, slot and entry
    # 12 B for a leaf, 16 B for an inner clique, 8 B for the root of the
    # schedule (any clique of degree one other than the root is a leaf)
    for cfg, kw in (("c1", {}), ("c2", {"n_cliques": 12}), ("c4", {"n_slots": 6})):
        inst = make_instance(cfg, 1, **kw)
        plan = jt.JunctionTreePlan.from_instance(inst)
        root = plan.query(jt.JT_Q_ROOT)
        deg = np.zeros(inst.n_cliques, int)
        for c, p in enumerate(inst.parent):
            if p >= 0:
                deg[c] += 1
                deg[p] += 1
        size = [int(np.prod(inst.card[inst.vars_of(c)])) for c in range(inst.n_cliques)]
        per_slot = sum(s * (8 if c == root else 12 if deg[c] == 1 else 16) for c, s in enumerate(size))
        n = max(1, inst.n_slots)
        assert plan.query(jt.JT_Q_ALG_BYTES, 0) == per_slot * n
        assert plan.query(jt.JT_Q_ALG_BYTES, 1) == per_slot
    single = jt.JunctionTreePlan(np.array([2, 3], np.int32), np.array([0, 2], np.int64), np.array([0, 1], np.int32),
                                 np.array([-1], np.int32), 1)
    assert single.query(jt.JT_Q_ALG_BYTES, 0) == 8 * 6
    with pytest.raises(jt.JTError):
        single.query(jt.JT_Q_ALG_BYTES, 2)
