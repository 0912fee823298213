#!/usr/bin/env python3
"""Benchmark of one junction-tree belief propagation on one MI355X.

A step is one full propagation (reset with evidence, collect, distribute,
posterior read-out of every clique left on the device) of a synthetic
large-clique junction tree: 64 cliques of 10 variables with 4 states
(1,048,576 FP32 entries per table), separators of 4-6 variables,
Dirichlet(1) rows over each table's innermost variable, 8 observed
variables.  Inputs are resident in HBM before the timed region.

Metric: BP table entries per second, counted as the numerator of the
paper's per-message cost (|phi_Xi| + |phi_Xk| per message, both sweeps).
Also reported: FP32 table bytes per second of the executed schedule, the
roofline of the dominant kernel (the streaming pass kernel) from per-launch
HIP events, the one-message-at-a-time schedule beside it, the error against
the FP64 oracle, and the oracle itself timed on the host cores.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c2": "large-clique tree: 64 cliques x 10 vars of card 4 (1,048,576 entries each), "
          "separators 4-6 vars, Dirichlet(1) rows, 8 observed vars, 1 query",
    "c3": "high-cardinality tree: 30 cliques x 3-4 vars of card 32/64 (up to 16.7M entries), "
          "separators 1-2 vars, Uniform(0,1), 4 observed vars, 1 query",
    "c4": "batched evidence: 200 cliques x 6-12 vars of card 2-3, separators 2-5 vars, "
          "256 evidence sets of 1-16 observed vars in one propagation",
    "c1": "tiny binary tree: 20 cliques x 5 binary vars, separators of 2 vars, 3 observed vars",
    "c5": "serving stream: 16 resident trees (total entries log-uniform 1e3..5e7, var cards 2-64), "
          "Poisson arrivals, uniform tree, 1-8 observed vars, all clique posteriors left on device",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="graph", choices=["graph", "fused", "plain"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="oracle leg: keep running whole propagations until this many seconds have passed")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="pick the schedule's shape choices by measurement first (auto: batched c4 only)")
    ap.add_argument("--tuning", default=None, help="JSON of jt_tuning fields, instead of autotuning")
    ap.add_argument("--queries", type=int, default=2000, help="c5: queries per arrival-rate run")
    ap.add_argument("--capacity", type=int, default=8, help="c5: evidence slots per resident tree")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="c5: HBM admission budget")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB FP32 tensor 5 times (the known-size reference kernel for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale)")
    return ap.parse_args()


COPY_BYTES = 256 << 20
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "jt_pass_kernel_{cfg}_traffic.json")


def calibrate_copy():
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 5}))


def measured_traffic(cfg, kernel, tuning=None):
    """HBM bytes per launch from the committed counter runs, or None when the
    kernel source or the schedule's shape choices differ from those the
    counters were taken with."""
    from paper_1202_3777_amd.rocprof_summary import kernel_source_hash
    f = TRAFFIC_FILE.format(cfg=cfg)
    if not os.path.exists(f):
        return None
    t = json.load(open(f))
    if t.get("source_sha256") != kernel_source_hash() or t.get("kernel") != kernel:
        return None
    if (tuning or {}) != t.get("tuning", {}):
        return None
    return t["traffic_bytes_per_launch"]


def serve_bench(args):
    """Served queries/s at saturation, then p50/p99 at 0.5x and 0.9x of it."""
    import torch
    from paper_1202_3777_amd import jt
    from paper_1202_3777_amd.instances import make_serving_trees
    from paper_1202_3777_amd.serve import Clock, Server, TreeExecutor, latency_stats, make_queries
    trees = make_serving_trees(seed=args.seed)
    log(f"[bench] c5: {len(trees)} trees, {sum(t.total_entries() for t in trees):,} entries resident")
    ex = [TreeExecutor(t, capacity=args.capacity, mode=args.mode if args.mode != "plain" else "plain") for t in trees]
    budget = int(args.budget_gib * 2 ** 30)

    def run(rate, n, seed):
        srv = Server(ex, budget_bytes=budget, clock=Clock(torch))
        qs = make_queries(trees, n, rate, seed=seed)
        done = srv.run(qs, max_seconds=240)
        st = latency_stats(done)
        st["batches"] = srv.n_batches
        st["mean_batch"] = float(np.mean(srv.batch_sizes)) if srv.batch_sizes else 0.0
        return st

    # warm-up: every tree, every slot count used below, graphs captured
    for e in ex:
        for k in range(1, args.capacity + 1):
            e.tree.propagate(e.mode, n_active=k)
    torch.cuda.synchronize()
    sat = run(None, args.queries, args.seed + 1)
    log(f"[bench] saturated: {sat}")
    lat = {}
    for frac in (0.5, 0.9):
        lat[str(frac)] = run(frac * sat["queries_per_s"], args.queries, args.seed + 2)
        log(f"[bench] rate {frac} x saturated: {lat[str(frac)]}")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # a bounded sample: queries of the same mix until --cpu-seconds have passed
        qs = make_queries(trees, 5000, None, seed=args.seed + 3)
        plans = {}
        t_plan = time.perf_counter()
        for i in range(len(trees)):
            plans[i] = oracle.Plan.from_instance(trees[i])
        t = time.perf_counter()
        n_q = 0
        for q in qs:
            plans[q.tree].run(trees[q.tree].potentials, q.ev_vars, q.ev_states, want_marginals=False)
            n_q += 1
            if time.perf_counter() - t >= args.cpu_seconds:
                break
        dt = time.perf_counter() - t
        cpu = {"value": n_q / dt, "unit": "queries/s", "cores": 1, "kind": "oracle",
               "sample": f"{n_q} queries of the same mix, FP64, single thread ({dt:.1f} s; mapping tables "
                         f"prebuilt in {t - t_plan:.1f} s)"}
        log(f"[bench] oracle {cpu['value']:.2f} queries/s")
    out = {
        "metric": "served queries/s (saturated), with p50/p99 latency at 0.5x and 0.9x of that rate",
        "value": sat["queries_per_s"], "unit": "queries/s", "n_gpus": 1, "steps": args.queries,
        "warmup": args.capacity, "ms_per_step": 1e3 / sat["queries_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded generator, no dataset)",
        "config": {"workload": f"c5: {WORKLOADS['c5']}", "seed": args.seed, "slots_per_tree": args.capacity,
                   "budget_gib": args.budget_gib, "schedule": args.mode, "parallelism": "single GPU"},
        "saturated": sat, "latency": lat, "roofline": None, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1202_3777_amd import jt
    from paper_1202_3777_amd.instances import make_instance

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.config == "c5":
        serve_bench(args)
        return
    log(f"[bench] generating {args.config} seed {args.seed}")
    inst = make_instance(args.config, args.seed)
    tuning, tune_table = {}, None
    if args.tuning:
        tuning = json.loads(args.tuning)
    elif args.autotune == "on" or (args.autotune == "auto" and args.config == "c4"):
        from paper_1202_3777_amd import tune
        log("[bench] autotuning the schedule's shape choices (untimed)")
        tuning, tune_table = tune.autotune(inst, mode=args.mode if args.mode != "plain" else "graph")
        for cand, ms in tune_table:
            log(f"[bench]   {json.dumps(cand):60s} {ms:.4f} ms")
        log(f"[bench] chosen: {json.dumps(tuning)}")
    tree = jt.JunctionTree.from_instance(inst, device="cuda:0", tuning=tuning)
    stream = tree.stream
    n_slots = tree.n_slots
    entries = 2 * tree.query(jt.JT_Q_ENTRIES_PER_SWEEP) * n_slots     # both sweeps, all slots
    bytes_fused = tree.query(jt.JT_Q_BYTES_FUSED)
    bytes_plain = tree.query(jt.JT_Q_BYTES_PLAIN)

    def timed(mode, steps, warmup):
        for _ in range(warmup):
            tree.propagate(mode)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(steps):
            tree.propagate(mode)
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / steps

    log(f"[bench] warmup {args.warmup}, timing {args.steps} steps, mode {args.mode}")
    ms = timed(args.mode, args.steps, args.warmup)
    log(f"[bench] {ms:.4f} ms per propagation")

    # dominant kernel: the streaming pass kernel, per-launch HIP events on the
    # library's stream, averaged over a few profiled propagations
    prof_mode = {"plain": "plain", "dataflow": "dataflow"}.get(args.mode, "fused")
    reps = 5
    pms, fms, nps = [], [], []
    for _ in range(reps):
        pm, fm, npass, nfin = tree.profile(prof_mode)
        pms.append(pm)
        fms.append(fm)
        nps.append(npass)
    pass_ms = float(np.mean(pms))
    n_pass = nps[0]
    table_bytes = bytes_plain if prof_mode == "plain" else bytes_fused
    kernel_name = "jt_dataflow_kernel" if prof_mode == "dataflow" else "jt_pass_kernel"
    avg_launch_ms = pass_ms / n_pass
    bytes_per_launch = table_bytes / n_pass
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    log(f"[bench] pass kernel: {n_pass} launches, {pass_ms:.4f} ms total, finalize {np.mean(fms):.4f} ms")

    # parity of this very run against the FP64 oracle, and the oracle timed
    worst = None
    cpu = None
    ms_plain = None
    if not args.no_plain and args.mode != "plain":
        ms_plain = timed("plain", max(3, args.steps // 10), 1)
        log(f"[bench] one-message-at-a-time schedule: {ms_plain:.4f} ms per propagation")
        tree.propagate(args.mode)
    if not args.no_cpu_baseline:
        import oracle
        log("[bench] oracle: building mapping tables (untimed)")
        oplan = oracle.Plan.from_instance(inst)
        slots = list(range(min(n_slots, 4)))
        # a bounded sample: whole propagations, cycling through the slots,
        # until --cpu-seconds have passed (the first slots' results are kept
        # for the error check below)
        kept = {}
        n_prop = 0
        t = time.perf_counter()
        while True:
            s = n_prop % n_slots
            res = oplan.run(inst.potentials, *inst.evidence[s])
            if s in slots and s not in kept:
                kept[s] = res
            del res
            n_prop += 1
            dt = time.perf_counter() - t
            if (dt >= args.cpu_seconds and len(kept) == len(slots)) or n_prop >= 100000:
                break
        refs = [kept[s] for s in slots]
        per_prop = dt / n_prop
        cpu = {"value": 2 * tree.query(jt.JT_Q_ENTRIES_PER_SWEEP) / per_prop, "unit": "entries/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{n_prop} full FP64 propagation(s) of the same tree, evidence sets cycled over "
                         f"{min(n_prop, n_slots)} slot(s) ({dt:.1f} s), mapping tables prebuilt, single thread"}
        log(f"[bench] oracle {per_prop:.2f} s per propagation")
        worst = 0.0
        lz_err = 0.0
        for s, res in zip(slots, refs):
            got, lz = tree.marginals_all(s)
            for c in range(inst.n_cliques):
                a = got[tree.table_off[c]:tree.table_off[c + 1]].astype(np.float64)
                b = oplan.marginal(res, c)
                worst = max(worst, float(np.max(np.abs(a - b)) / np.max(np.abs(b))))
            lz_err = max(lz_err, abs(lz - res["logz"]))
        log(f"[bench] max rel err vs FP64 {worst:.3e}, |dlogZ| {lz_err:.3e}")

    value = entries / (ms * 1e-3)
    out = {
        "metric": "BP table entries/s (collect + distribute, sum of |phi_Xi|+|phi_Xk| per message)",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator, no dataset)",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "seed": args.seed,
                   "n_slots": n_slots, "schedule": args.mode, "parallelism": "single GPU",
                   "tuning": tuning or "defaults", "lanes": tree.query(jt.JT_Q_N_LANES),
                   "autotune_ms": None if tune_table is None else [[c, round(ms, 4)] for c, ms in tune_table]},
        "hbm_gbs_table_bytes": (bytes_fused if args.mode != "plain" else bytes_plain) / (ms * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.config, kernel_name, tuning),
                     "kernel": kernel_name, "launches_per_step": n_pass,
                     "avg_launch_us": avg_launch_ms * 1e3, "bytes_per_launch": bytes_per_launch},
        "plain_sweep": None if ms_plain is None else {
            "ms_per_step": ms_plain, "value": entries / (ms_plain * 1e-3), "unit": "entries/s",
            "launches_per_step": tree.query(jt.JT_Q_N_LAUNCHES_PLAIN)},
        "max_rel_err_vs_fp64": worst,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
