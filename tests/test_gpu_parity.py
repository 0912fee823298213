"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Tolerance (FP32 tables, FP64 log-normalizer): for every clique,
    ||P_gpu - P_oracle||_inf / ||P_oracle||_inf <= 1e-5
and |log Z_gpu - log Z_oracle| <= 1e-5 * max(1, |log Z_oracle|).
Beside it, the elementwise relative error |P_gpu - P_oracle| / P_oracle over
the entries with P_oracle >= 1e-3 * max P_oracle of their clique is printed
and held to 1e-4 (each such entry is a product of O(depth) rounded ratios
and scales, a few hundred FP32 ulps at most).  The errors against FP64 are
printed for every case.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1202_3777_amd.instances import from_arrays, make_instance

pytestmark = pytest.mark.gpu

TOL = 1e-5
ELEM_TOL = 1e-4


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_3777_amd import jt
    return jt


def compare(tree, plan, inst, slot, res, label=""):
    """Compare one slot of a propagated tree with an oracle result."""
    got, lz = tree.marginals_all(slot)
    worst, elem = errors(got, tree.table_off, plan, res, inst.n_cliques)
    dlz = abs(lz - res["logz"])
    print(f"[parity] {label} slot={slot} max_rel_err={worst:.3e} elem_rel_err={elem:.3e} dlogZ={dlz:.3e} "
          f"logZ={res['logz']:.6f}")
    assert worst <= TOL, (label, slot, worst)
    assert elem <= ELEM_TOL, (label, slot, elem)
    assert dlz <= TOL * max(1.0, abs(res["logz"])), (label, slot, dlz)
    return worst


def errors(got, table_off, plan, res, n_cliques):
    """(normwise, elementwise) relative errors of packed posteriors against
    an oracle result: max over cliques of ||a-b||_inf/||b||_inf, and max
    |a-b|/b over the entries b >= 1e-3 * max(b) of each clique."""
    worst = elem = 0.0
    for c in range(n_cliques):
        a = got[table_off[c]:table_off[c + 1]].astype(np.float64)
        b = plan.marginal(res, c)
        mb = np.max(np.abs(b))
        worst = max(worst, float(np.max(np.abs(a - b)) / mb))
        big = b >= 1e-3 * mb
        elem = max(elem, float(np.max(np.abs(a[big] - b[big]) / b[big])))
    return worst, elem


def run_case(inst, modes=("fused", "graph", "plain"), slots=None, n_slots=None):
    jt = _gpu()
    plan = oracle.Plan.from_instance(inst)
    tree = jt.JunctionTree.from_instance(inst, n_slots=n_slots)
    slots = range(tree.n_slots) if slots is None else slots
    refs = {s: plan.run(inst.potentials, *inst.evidence[s]) for s in slots}
    for mode in modes:
        tree.propagate(mode)
        for s in slots:
            compare(tree, plan, inst, s, refs[s], f"{inst.name}/{mode}")
    return tree, plan, refs


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c1_all_modes(seed):
    run_case(make_instance("c1", seed))


def test_c1_truncated_bruteforce_shape():
    # the small trees the oracle is pinned on by full-joint enumeration
    for seed in range(3):
        run_case(make_instance("c1", seed, n_cliques=7, n_obs=(0, 3)), modes=("fused", "plain"))


def test_c2_full_size():
    run_case(make_instance("c2", 0))


def test_c2_conditional_partition_function():
    jt = _gpu()
    inst = make_instance("c2", 3, conditional=True, n_cliques=12, n_obs=(0, 0))
    tree = jt.JunctionTree.from_instance(inst)
    tree.propagate("graph")
    _, lz = tree.marginals_all(0)
    print(f"[parity] c2-conditional logZ={lz:.3e}")
    assert abs(lz) < 1e-4


def test_c3_full_size():
    run_case(make_instance("c3", 0), modes=("fused", "plain"))


def test_c3_other_seed_ragged():
    run_case(make_instance("c3", 1, n_cliques=12), modes=("graph",))


def test_c4_batched_slots():
    inst = make_instance("c4", 0, n_slots=8)
    run_case(inst, modes=("fused", "graph"))


C4_FALLBACK_TUNING = {"target_blocks": 10240}


def bench_tuning(inst):
    """The shape choice the benchmark runs this tree with: the autotuner's
    cached choice for this GPU and kernel source, else a fixed one."""
    import torch
    from paper_1202_3777_amd import tune
    t = tune.cache_lookup(tune.shape_key(inst, device_name=torch.cuda.get_device_name(0)))
    return t if t is not None else C4_FALLBACK_TUNING


def test_c4_full_batch_every_slot():
    # the 256-slot batch in the launch configuration the benchmark times
    # (graph schedule, autotuned shape, shared evidence-free collect
    # messages): every slot against the oracle
    jt = _gpu()
    inst = make_instance("c4", 0)
    plan = oracle.Plan.from_instance(inst)
    tuning = bench_tuning(inst)
    print(f"[parity] c4 shape choice {tuning}")
    tree = jt.JunctionTree.from_instance(inst, tuning=tuning)
    tree.propagate("graph")
    assert tree.query(jt.JT_Q_LAST_SHARED) == 1
    passes = tree.query(jt.JT_Q_LAST_COLLECT_PASSES)
    print(f"[parity] c4 collect passes {passes} of {inst.n_cliques * 256} (clique, slot) pairs")
    assert passes < inst.n_cliques * 256 // 2
    for s in range(inst.n_slots):
        compare(tree, plan, inst, s, plan.run(inst.potentials, *inst.evidence[s]), "c4/graph/all-slots")


def test_c4_full_batch_repeats_bit_identical():
    # the benchmark's configuration propagated again and again: graph replays
    # and launch-by-launch propagations (one-slot and multi-slot launches on
    # two streams, levels not joined in between) give the same bits every
    # time -- a race between the streams would show as a difference
    jt = _gpu()
    import torch
    inst = make_instance("c4", 0)
    tree = jt.JunctionTree.from_instance(inst, tuning=bench_tuning(inst))
    n, tot = inst.n_slots, int(tree.table_off[-1])

    def run(mode):
        tree.propagate(mode)
        post = torch.empty(n * tot, dtype=torch.float32, device="cuda:0")
        lz = torch.empty(n, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()   # allocated before the tree's stream writes them
        jt.jt_read_out(tree.handle, 0, n, post.data_ptr(), lz.data_ptr())
        torch.cuda.synchronize()
        return post, lz

    ref, rlz = run("graph")
    assert bool(torch.isfinite(ref).all()) and bool((ref >= 0).all())
    for k, mode in enumerate(("graph", "graph", "fused", "fused", "graph")):
        print(f"[parity] c4 repeat {k} ({mode})", flush=True)
        p, lz = run(mode)
        assert torch.equal(p, ref) and torch.equal(lz, rlz), (k, mode)
        del p, lz


def test_c4_shared_edge_cases():
    # slots without any evidence (every collect message shared), a slot
    # observing one variable of the center clique, a batch where sharing is
    # not worth it (one active slot), and both fused and graph schedules
    jt = _gpu()
    inst = make_instance("c4", 3, n_slots=12, n_obs=(0, 4))
    p0 = jt.JunctionTreePlan.from_instance(inst)
    root = p0.query(jt.JT_Q_ROOT)
    center_var = int(inst.vars_of(root)[0])
    inst.evidence[1] = (np.zeros(0, np.int32), np.zeros(0, np.int32))
    inst.evidence[2] = (np.asarray([center_var], np.int32), np.asarray([1], np.int32))
    plan = oracle.Plan.from_instance(inst)
    refs = {s: plan.run(inst.potentials, *inst.evidence[s]) for s in range(inst.n_slots)}
    tree = jt.JunctionTree.from_instance(inst)
    for mode in ("fused", "graph"):
        tree.propagate(mode)
        assert tree.query(jt.JT_Q_LAST_SHARED) == 1
        for s in range(inst.n_slots):
            compare(tree, plan, inst, s, refs[s], f"c4-shared/{mode}")
    full = [tree.marginals_all(s) for s in range(inst.n_slots)]
    tree.propagate("graph", n_active=1)
    assert tree.query(jt.JT_Q_LAST_SHARED) == 0
    a, la = tree.marginals_all(0)
    assert np.array_equal(a, full[0][0]) and la == full[0][1]
    # new evidence in one slot: the schedule follows it (a new set of grids)
    tree.set_evidence(5, [center_var], [0])
    tree.propagate("graph")
    compare(tree, plan, inst, 5, plan.run(inst.potentials, [center_var], [0]), "c4-shared/changed")
    for s in (0, 4, 6):
        b, lb = tree.marginals_all(s)
        assert np.array_equal(b, full[s][0]) and lb == full[s][1]


def test_autotuner_candidates_full_size():
    # every shape choice the autotuner may hand to the benchmark: the c4
    # 256-slot batch (sampled slots) and the c2 tree, each against the oracle
    jt = _gpu()
    from paper_1202_3777_amd.tune import DEFAULT_CANDIDATES
    for cfg, slots in (("c4", [0, 201]), ("c2", [0])):
        inst = make_instance(cfg, 0)
        plan = oracle.Plan.from_instance(inst)
        refs = {s: plan.run(inst.potentials, *inst.evidence[s]) for s in slots}
        for cand in DEFAULT_CANDIDATES:
            tree = jt.JunctionTree.from_instance(inst, tuning=cand)
            tree.propagate("graph")
            for s in slots:
                compare(tree, plan, inst, s, refs[s], f"{inst.name}/graph/{cand}")
            del tree


def test_odd_shapes():
    # prime cardinality above the tile limit (one-entry tiles), cardinality 1,
    # cardinality-3 tables (scalar loads), an empty separator, a single-clique
    # tree, evidence on split digits
    cases = [
        from_arrays([257, 2, 1, 3, 5, 7], [[0, 1], [1, 2, 3], [3, 4, 5], [5]], [-1, 0, 1, 2], seed=1,
                    evidence=[([0, 4], [200, 3])]),
        from_arrays([2, 3, 4], [[0, 1], [2]], [-1, 0], seed=2, evidence=[([2], [1])]),
        from_arrays([3, 5, 7], [[0, 1, 2]], [-1], seed=3, evidence=[([1], [4])]),
        from_arrays([64, 64, 32, 3], [[0, 1, 2], [2, 3, 0]], [-1, 0], seed=4,
                    evidence=[([1, 3], [17, 2])]),
        from_arrays([3] * 9, [[0, 1, 2, 3, 4, 5], [5, 6, 7, 8, 0]], [-1, 0], seed=5,
                    evidence=[([6], [1])]),
        # a clique with 12 children: gathers past the register ones, staged in LDS
        from_arrays([2] * 30, [[0, 1, 2, 3, 4, 5]] + [[k % 6, (k + 1) % 6, 6 + 2 * k, 7 + 2 * k] for k in range(12)],
                    [-1] + [0] * 12, seed=6, evidence=[([7, 20, 2], [1, 0, 1])]),
        # 24 children of a 256-entry clique: too many to stage, read tile by tile
        from_arrays([2] * 56, [list(range(8))] + [[k % 8, (k + 3) % 8, 8 + 2 * k, 9 + 2 * k] for k in range(24)],
                    [-1] + [0] * 24, seed=7, evidence=[([9, 30, 1], [0, 1, 1])]),
    ]
    for inst in cases:
        run_case(inst)


def test_hub_with_chained_prepasses():
    # a hub whose 14 children finish at heights 0..6: its messages are
    # absorbed in three chained pre-passes before the hub's own pass; four
    # evidence sets batched (one evidence-free, so the hub's collect passes
    # are shared by some sets and not by others), then each set alone
    from shapes import hub_with_chains
    inst, _ = hub_with_chains(0)
    run_case(inst)
    for ev in inst.evidence:
        run_case(dataclasses.replace(inst, evidence=[ev]), modes=("fused", "plain"))


def test_paired_tiles():
    # 108-entry tiles streamed two per wave load: 243 tiles (odd, a half-wave
    # idles on each chunk's last step), evidence zeroing whole tiles and
    # masking positions, six sets batched (two share multi-slot passes),
    # then each set alone, and the batched bits equal the lone ones
    from shapes import paired_tiles
    inst = paired_tiles(0)
    batched, _, _ = run_case(inst)
    batched.propagate("fused")
    for s, ev in enumerate(inst.evidence):
        lone, _, _ = run_case(dataclasses.replace(inst, evidence=[ev]), modes=("plain", "fused"))
        a, la = batched.marginals_all(s)
        b, lb = lone.marginals_all(0)
        assert np.array_equal(a, b) and la == lb, s


def test_zero_evidence():
    jt = _gpu()
    card = [2, 2, 3]
    t0 = np.array([0.5, 0.0, 0.25, 0.0], dtype=np.float32)
    t1 = np.array([0.2, 0.3, 0.5, 0.1, 0.6, 0.3], dtype=np.float32)
    inst = from_arrays(card, [[0, 1], [1, 2]], [-1, 0], potentials=np.concatenate([t0, t1]),
                       evidence=[([2], [1])])
    tree, plan, refs = run_case(inst)     # a zero separator entry: 0/0 rule, no NaN
    got, _ = tree.marginals_all(0)
    assert np.all(np.isfinite(got))
    for mode in ("fused", "graph", "plain"):
        tree.set_evidence(0, [1], [1])     # probability zero
        tree.propagate(mode)
        with pytest.raises(jt.JTError) as ei:
            tree.marginal(0, 0)
        assert ei.value.code == jt.JT_E_ZERO_EVIDENCE


def test_determinism_and_idempotence():
    jt = _gpu()
    inst = make_instance("c2", 1, n_cliques=10)
    tree = jt.JunctionTree.from_instance(inst)
    tree.propagate("fused")
    a, la = tree.marginals_all(0)
    tree.propagate("fused")
    b, lb = tree.marginals_all(0)
    tree.propagate("graph")
    c, lc = tree.marginals_all(0)
    assert np.array_equal(a, b) and la == lb
    assert np.array_equal(a, c) and la == lc
    # new evidence, then back: results follow the evidence, and come back bit-identical
    plan = oracle.Plan.from_instance(inst)
    tree.set_evidence(0, [3, 40], [1, 2])
    tree.propagate("graph")
    compare(tree, plan, inst, 0, plan.run(inst.potentials, [3, 40], [1, 2]), "c2-evidence-change")
    tree.set_evidence(0, *inst.evidence[0])
    tree.propagate("graph")
    d, ld = tree.marginals_all(0)
    assert np.array_equal(a, d) and la == ld


def test_batched_slot_equals_single():
    jt = _gpu()
    inst = make_instance("c4", 5, n_slots=6)
    batch = jt.JunctionTree.from_instance(inst)
    batch.propagate("graph")
    for s in (0, 3, 5):
        single = jt.JunctionTree(inst.card, inst.clique_off, inst.clique_vars, inst.parent, inst.potentials, 1)
        single.set_evidence(0, *inst.evidence[s])
        single.propagate("graph")
        a, la = batch.marginals_all(s)
        b, lb = single.marginals_all(0)
        assert np.array_equal(a, b) and la == lb


def test_profile_reports_launches():
    jt = _gpu()
    inst = make_instance("c1", 0)
    tree = jt.JunctionTree.from_instance(inst)
    pm, fm, npass, nfin = tree.profile("fused")
    assert npass == tree.query(jt.JT_Q_N_LAUNCHES_FUSED) and pm > 0 and nfin == 0
    plan = oracle.Plan.from_instance(inst)
    compare(tree, plan, inst, 0, plan.run(inst.potentials, *inst.evidence[0]), "c1-profiled")


DATAFLOW_SKIP = ("the persistent dataflow launch did not complete on its first GPU run (c1, seed 0); "
                 "no cause has been shown, so the schedule is disabled and stays off the GPU until one is")


@pytest.mark.skip(reason=DATAFLOW_SKIP)
def test_dataflow_schedule_parity():
    for inst in (make_instance("c1", 0), make_instance("c3", 1, n_cliques=12), make_instance("c4", 0, n_slots=8)):
        run_case(inst, modes=("dataflow",))


@pytest.mark.skip(reason=DATAFLOW_SKIP)
def test_dataflow_bit_identical_to_levels():
    jt = _gpu()
    inst = make_instance("c2", 1, n_cliques=10)
    tree = jt.JunctionTree.from_instance(inst)
    tree.propagate("graph")
    a, la = tree.marginals_all(0)
    tree.propagate("dataflow")
    e, le = tree.marginals_all(0)
    assert np.array_equal(a, e) and la == le


def test_dataflow_is_refused():
    jt = _gpu()
    tree = jt.JunctionTree.from_instance(make_instance("c1", 0))
    with pytest.raises(jt.JTError) as ei:
        tree.propagate("dataflow")
    assert ei.value.code == jt.JT_E_ARG


def test_propagate_active_prefix():
    jt = _gpu()
    inst = make_instance("c4", 7, n_slots=4)
    tree = jt.JunctionTree.from_instance(inst)
    tree.propagate("graph")
    full = [tree.marginals_all(s) for s in range(4)]
    for mode in ("fused", "graph"):
        tree.propagate(mode, n_active=2)
        for s in range(2):
            a, la = tree.marginals_all(s)
            assert np.array_equal(a, full[s][0]) and la == full[s][1]
        with pytest.raises(jt.JTError) as ei:
            tree.marginals_all(2)
        assert ei.value.code == jt.JT_E_STATE
    with pytest.raises(jt.JTError):
        tree.propagate("graph", n_active=5)


def test_paper_schedule_parity_and_layouts():
    # the paper's own kernel design (one thread per separator entry over
    # explicit mapping lists, one message at a time): against the oracle,
    # and bit-identical between the naive and interleaved layouts, across
    # block sizes and between eager launches and a captured graph
    jt = _gpu()
    cases = [make_instance("c1", 0), make_instance("c4", 2, n_slots=3), make_instance("c2", 1, n_cliques=6),
             make_instance("c3", 1, n_cliques=6),
             from_arrays([257, 2, 1, 3, 5, 7], [[0, 1], [1, 2, 3], [3, 4, 5], [5]], [-1, 0, 1, 2], seed=1,
                         evidence=[([0, 4], [200, 3])]),
             from_arrays([2, 3, 4], [[0, 1], [2]], [-1, 0], seed=2, evidence=[([2], [1])])]
    for inst in cases:
        plan = oracle.Plan.from_instance(inst)
        tree = jt.JunctionTree.from_instance(inst)
        tree.paper_bind("naive", 64)
        tree.propagate("paper")
        first = []
        for s in range(tree.n_slots):
            compare(tree, plan, inst, s, plan.run(inst.potentials, *inst.evidence[s]), f"{inst.name}/paper-naive")
            first.append(tree.marginals_all(s))
        for layout, tpb, mode in (("interleaved", 256, "paper"), ("interleaved", 32, "paper_graph"),
                                  ("naive", 512, "paper_graph")):
            tree.paper_bind(layout, tpb)
            tree.propagate(mode)
            for s in range(tree.n_slots):
                a, la = tree.marginals_all(s)
                assert np.array_equal(a, first[s][0]) and la == first[s][1], (inst.name, layout, tpb, mode)


def test_merged_small_separators():
    # the paper's future work: small separators merged away; the caller's
    # cliques' posteriors (marginalized from the merged cliques on the
    # device) against the oracle on the unmerged tree
    jt = _gpu()
    cases = [(make_instance("c1", 0), (4, 4096)), (make_instance("c1", 1), (4, 1 << 16)),
             (make_instance("c4", 2, n_slots=5), (8, 1 << 16)),
             (make_instance("c3", 1, n_cliques=8), (32, 1 << 22)),
             (from_arrays([2, 3, 4], [[0, 1], [2]], [-1, 0], seed=2, evidence=[([2], [1])]), (1, 64))]
    for inst, merge in cases:
        plan = oracle.Plan.from_instance(inst)
        tree = jt.JunctionTree.from_instance(inst, merge=merge)
        print(f"[merged] {inst.name}: {inst.n_cliques} cliques -> {tree.n_compiled}")
        for mode in ("fused", "graph", "plain"):
            tree.propagate(mode)
            for s in range(tree.n_slots):
                compare(tree, plan, inst, s, plan.run(inst.potentials, *inst.evidence[s]), f"{inst.name}/merged/{mode}")
        one, _ = tree.marginal(0, inst.n_cliques - 1)
        allm, _ = tree.marginals_all(0)
        assert np.array_equal(one, allm[tree.table_off[-2]:tree.table_off[-1]])
