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
    ap.add_argument("--no-plain", action="store_true")
    return ap.parse_args()


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
    log(f"[bench] generating {args.config} seed {args.seed}")
    inst = make_instance(args.config, args.seed)
    tree = jt.JunctionTree.from_instance(inst, device="cuda:0")
    stream = tree.stream
    n_slots = tree.n_slots
    entries = 2 * tree.query(jt.JT_Q_ENTRIES_PER_SWEEP) * n_slots     # both sweeps, all slots
    bytes_fused = tree.query(jt.JT_Q_BYTES_FUSED)
    bytes_plain = tree.query(jt.JT_Q_BYTES_PLAIN) * n_slots

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
    prof_mode = "plain" if args.mode == "plain" else "fused"
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
        t = time.perf_counter()
        refs = [oplan.run(inst.potentials, *inst.evidence[s]) for s in slots]
        dt = time.perf_counter() - t
        per_prop = dt / len(slots)
        cpu = {"value": 2 * tree.query(jt.JT_Q_ENTRIES_PER_SWEEP) / per_prop, "unit": "entries/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{len(slots)} full FP64 propagation(s) of the same tree and evidence "
                         f"({dt:.1f} s), mapping tables prebuilt, single thread"}
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
                   "n_slots": n_slots, "schedule": args.mode, "parallelism": "single GPU"},
        "hbm_gbs_table_bytes": (bytes_fused if args.mode != "plain" else bytes_plain) / (ms * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "jt_pass_kernel", "launches_per_step": n_pass,
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
