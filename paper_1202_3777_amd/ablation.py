"""The paper's own kernel design against the tiled engine, on synthetic trees.

    python -m paper_1202_3777_amd.ablation [--quick] [--out FILE.json]

Runs on one GPU and prints one JSON object (also written to --out):

  * block_size  -- the paper's Fig. 5: time of one propagation with the
    paper's kernels (one thread per separator entry, interleaved mapping
    lists, graph-replayed) against the threads per block, on a tree with
    large separators (the large-clique tree, 12 cliques) and one with small
    ones (the batched tree's shape, one evidence set);
  * layout      -- Fig. 8: naive against interleaved mapping lists;
  * sep_sweep   -- Fig. 6: trees whose separators hold 1..12 binary
    variables; the oracle (sequential FP64 on the host) over the paper's
    kernels and over the tiled engine, against the average separator size;
  * overhead    -- Fig. 7's question asked of this GPU: the time of one
    propagation launched launch by launch against the same launches replayed
    from a captured graph (the difference is the launch cost the graph
    removes), for the paper's schedule and the tiled one; the kernels' own
    busy time comes from a rocprofv3 kernel trace of the same command;
  * margin      -- the tiled engine's speedup over the paper's kernels;
  * merge       -- the paper's future work (Sec. 5): the same trees with
    their small separators merged away, time per propagation against the
    unmerged tree (the caller's clique posteriors read out in both).

Every timed propagation is checked against the oracle first.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def _time(torch, tree, mode, reps):
    tree.propagate(mode)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(tree.stream)
    for _ in range(reps):
        tree.propagate(mode)
    b.record(tree.stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _check(tree, inst, plan, res):
    got, lz = tree.marginals_all(0)
    worst = 0.0
    for c in range(inst.n_cliques):
        a = got[tree.table_off[c]:tree.table_off[c + 1]].astype(np.float64)
        ref = plan.marginal(res, c)
        worst = max(worst, float(np.max(np.abs(a - ref)) / np.max(ref)))
    if worst > 1e-5 or abs(lz - res["logz"]) > 1e-5 * max(1.0, abs(res["logz"])):
        raise RuntimeError(f"{inst.name}: parity failed ({worst:.3e})")
    return worst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--sections", default="block_size,sep_sweep,overhead,merge")
    args = ap.parse_args()
    sections = set(args.sections.split(","))
    import torch

    import oracle
    from paper_1202_3777_amd import jt
    from paper_1202_3777_amd.instances import make_instance, make_separator_sweep

    out = {"device": torch.cuda.get_device_name(0)}
    reps = args.reps

    def tree_of(inst):
        t = jt.JunctionTree.from_instance(inst, n_slots=1)
        return t

    # Fig. 5 and Fig. 8
    trees = {} if "block_size" not in sections else {"large separators (12 cliques of the large-clique tree)": make_instance("c2", 0, n_cliques=12),
             "small separators (the batched tree, one evidence set)": make_instance("c4", 0, n_slots=1)}
    tpbs = [16, 32, 64, 128, 256, 512] if not args.quick else [32, 256]
    out["block_size"], out["layout"] = {}, {}
    for name, inst in trees.items():
        plan = oracle.Plan.from_instance(inst)
        res = plan.run(inst.potentials, *inst.evidence[0])
        t = tree_of(inst)
        row = {}
        for tpb in tpbs:
            t.paper_bind("interleaved", tpb)
            row[tpb] = _time(torch, t, "paper_graph", reps)
            _check(t, inst, plan, res)
        out["block_size"][name] = row
        best = min(row, key=row.get)
        t.paper_bind("naive", best)
        naive = _time(torch, t, "paper_graph", reps)
        _check(t, inst, plan, res)
        out["layout"][name] = {"threads_per_block": best, "naive_ms": naive, "interleaved_ms": row[best],
                               "interleaved_speedup": naive / row[best]}
        print(name, json.dumps(row), json.dumps(out["layout"][name]), flush=True)
        del t

    # Fig. 6: speedup against the average separator size
    out["sep_sweep"] = []
    for s in (range(1, 13) if not args.quick else (2, 6, 10)) if "sep_sweep" in sections else ():
        inst = make_separator_sweep(s, seed=s)
        plan = oracle.Plan.from_instance(inst)
        # one untimed run, then the median of up to 50 timed ones (0.5 s)
        res = plan.run(inst.potentials, *inst.evidence[0])
        laps = []
        t_end = time.perf_counter() + 0.5
        while len(laps) < 50 and (not laps or time.perf_counter() < t_end):
            t0 = time.perf_counter()
            res = plan.run(inst.potentials, *inst.evidence[0])
            laps.append(time.perf_counter() - t0)
        cpu_ms = float(np.median(laps)) * 1e3
        t = tree_of(inst)
        t.paper_bind("interleaved", 64)
        paper_ms = _time(torch, t, "paper_graph", reps)
        _check(t, inst, plan, res)
        tiled_ms = _time(torch, t, "graph", reps)
        _check(t, inst, plan, res)
        row = {"sep_vars": s, "avg_sep_entries": 2 ** s, "avg_clique_entries": 2 ** (s + 4),
               "cpu_ms": cpu_ms, "paper_ms": paper_ms, "tiled_ms": tiled_ms,
               "paper_speedup": cpu_ms / paper_ms, "tiled_speedup": cpu_ms / tiled_ms}
        out["sep_sweep"].append(row)
        print(json.dumps(row), flush=True)
        del t

    # Fig. 7: launch-by-launch against graph replay
    out["overhead"] = {}
    for name, inst in (("small separators", make_instance("c4", 0, n_slots=1)),
                       ("large separators", make_instance("c2", 0, n_cliques=12))) if "overhead" in sections else ():
        t = tree_of(inst)
        t.paper_bind("interleaved", 64)
        row = {"paper_eager_ms": _time(torch, t, "paper", reps), "paper_graph_ms": _time(torch, t, "paper_graph", reps),
               "tiled_eager_ms": _time(torch, t, "fused", reps), "tiled_graph_ms": _time(torch, t, "graph", reps),
               "paper_launches": 1 + 3 * 2 * (inst.n_cliques - 1) + 3,
               "tiled_launches": t.query(jt.JT_Q_N_LAUNCHES_FUSED)}
        row["paper_launch_share"] = 1.0 - row["paper_graph_ms"] / row["paper_eager_ms"]
        out["overhead"][name] = row
        out.setdefault("margin", {})[name] = row["paper_graph_ms"] / row["tiled_graph_ms"]
        print(name, json.dumps(row), flush=True)
        del t
    # Sec. 5: merging small separators
    out["merge"] = {}
    if "merge" in sections:
        cases = [("tiny binary tree (20 cliques of 32 entries)", make_instance("c1", 0), [(4, 1024), (4, 1 << 14)]),
                 ("batched tree's shape, one evidence set", make_instance("c4", 0, n_slots=1),
                  [(8, 1 << 17), (16, 1 << 18)])]
        for name, inst, bounds in cases:
            plan = oracle.Plan.from_instance(inst)
            res = plan.run(inst.potentials, *inst.evidence[0])
            t = jt.JunctionTree.from_instance(inst, n_slots=1)
            row = {"unmerged": {"cliques": inst.n_cliques, "launches": t.query(jt.JT_Q_N_LAUNCHES_FUSED),
                                "ms": _time(torch, t, "graph", max(reps, 20))}}
            _check(t, inst, plan, res)
            del t
            for ms_, me in bounds:
                t = jt.JunctionTree.from_instance(inst, n_slots=1, merge=(ms_, me))
                row[f"max_sep {ms_}, max_entries {me}"] = {
                    "cliques": t.n_compiled, "launches": t.query(jt.JT_Q_N_LAUNCHES_FUSED),
                    "ms": _time(torch, t, "graph", max(reps, 20))}
                _check(t, inst, plan, res)
                del t
            out["merge"][name] = row
            print(name, json.dumps(row), flush=True)
    s = json.dumps(out)
    print(s, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
