#!/usr/bin/env python3
"""Benchmark of junction-tree belief propagation on one MI355X.

Default workload (the largest single-GPU one): one batched propagation of
256 evidence sets over a 200-clique junction tree (6-12 variables of
cardinality 2-3 per clique, separators of 2-5 variables, Uniform(0.1, 1)
potentials, 1-16 observed variables per set).  A step is one full
propagation of all 256 sets: reset with evidence, collect, distribute, every
clique's posterior of every set written to the device.  Inputs are resident
in HBM before the timed region; the evidence-free collect messages are
recomputed inside every step.

Metric: BP table entries per second, counted as the numerator of the
paper's per-message cost (|phi_Xi| + |phi_Xk| per message, both sweeps,
every evidence set).  Also reported:
  * roofline of the dominant kernel (the streaming pass kernels -- the
    one-slot and the multi-slot variant of one pass -- the only kernels of
    a propagation): the algorithmic FP32 table bytes of a fused propagation
    (per clique, evidence set and entry: 12 B for a leaf, 16 B for an inner
    clique, 8 B for the root) over the graph-replayed launch time, HIP events
    on the tree's stream around the timed steps, against the 8 TB/s HBM peak
    and a copy kernel measured in the same run; beside it the bytes the
    executed schedule moved (shared evidence-free collect tables make that
    fewer) and the HBM traffic the counters measured;
  * the one-query-at-a-time GPU sweep (the paper's schedule: one message at a
    time, each evidence set alone) on the same 256 sets;
  * the error of every set against the FP64 oracle;
  * the oracle timed on the host cores (single thread, and all cores);
  * the serving stream (16 resident trees, Poisson arrivals): queries/s and
    p50/p99 latency beside the one-query-at-a-time GPU sweep.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c4": "batched evidence: 200 cliques x 6-12 vars of card 2-3, separators 2-5 vars, Uniform(0.1,1), "
          "256 evidence sets of 1-16 observed vars in one propagation",
    "c2": "large-clique tree: 64 cliques x 10 vars of card 4 (1,048,576 entries each), "
          "separators 4-6 vars, Dirichlet(1) rows, 8 observed vars, 1 query",
    "c3": "high-cardinality tree: 30 cliques x 3-4 vars of card 32/64 (up to 16.7M entries), "
          "separators 1-2 vars, Uniform(0,1), 4 observed vars, 1 query",
    "c1": "tiny binary tree: 20 cliques x 5 binary vars, separators of 2 vars, 3 observed vars",
    "c5": "serving stream: 16 resident trees (total entries log-uniform 1e3..5e7, var cards 2-64), "
          "Poisson arrivals, uniform tree, 1-8 observed vars, every clique posterior read out per query",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="graph", choices=["graph", "fused", "plain"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="oracle legs: keep running whole propagations until this many seconds have passed")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg of the default run")
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="auto: the cached choice for this shape class, else tune (batched config only); "
                         "on: always tune (and store the choice in the cache)")
    ap.add_argument("--tuning", default=None, help="JSON of jt_tuning fields, instead of autotuning")
    ap.add_argument("--queries", type=int, default=2000, help="serving: queries per arrival-rate run")
    ap.add_argument("--capacity", type=int, default=16, help="serving: evidence slots per lane of a resident tree")
    ap.add_argument("--serve-lanes", type=int, default=1,
                    help="serving: handles (workspace + stream) per resident tree; the GPU has few hardware queues, "
                         "and more streams queue batches of small trees behind those of large ones")
    ap.add_argument("--serve-mode", default="fused", choices=["fused", "graph"],
                    help="serving: schedule of the batched propagations (fused launches by default: every batch "
                         "has new evidence, so its listed launches' grids change and a graph would be re-captured)")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serving: HBM admission budget")
    ap.add_argument("--ceilings", action="store_true",
                    help="only measure this GPU's streaming ceilings (fill, read, copy, scale-in-place kernels of "
                         "torch, 256 MiB and 2 GiB) and print them as one JSON line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB FP32 tensor 5 times (the known-size reference kernel for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale)")
    return ap.parse_args()


COPY_BYTES = 256 << 20
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "jt_pass_{cfg}_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def calibrate_copy():
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 5}))


def copy_ceiling_gbs(torch, nbytes=2 << 30, reps=10):
    """HBM rate of a plain device copy (bytes read + bytes written per second)."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def ceilings():
    """HBM rates of plain streaming kernels: write-only (fill), read-only
    (sum), read+write (copy, in-place-free scale); bytes moved / time."""
    import torch
    out = {}
    for nb in (256 << 20, 2 << 30):
        a = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)

        def rate(fn, moved, reps=20):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return moved / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9

        out[f"{nb >> 20} MiB"] = {"fill_write_gbs": rate(lambda: b.fill_(1.5), nb),
                                  "sum_read_gbs": rate(lambda: a.sum(), nb),
                                  "copy_gbs": rate(lambda: b.copy_(a), 2 * nb),
                                  "scale_gbs": rate(lambda: torch.mul(a, 1.0001, out=b), 2 * nb)}
        del a, b
        torch.cuda.empty_cache()
    print(json.dumps({"ceilings": out, "device": torch.cuda.get_device_name(0)}))


def measured_traffic(cfg, kernel, tuning=None):
    """HBM bytes per launch from the committed counter runs, or None when the
    kernel source, the planner's source or the schedule's shape choices
    differ from those the counters were taken with."""
    from paper_1202_3777_amd.rocprof_summary import kernel_source_hash, plan_source_hash
    f = TRAFFIC_FILE.format(cfg=cfg)
    if not os.path.exists(f):
        return None
    t = json.load(open(f))
    if t.get("source_sha256") != kernel_source_hash() or t.get("kernel") != kernel:
        return None
    if t.get("plan_sha256") != plan_source_hash():
        return None
    if (tuning or {}) != t.get("tuning", {}):
        return None
    return t["traffic_bytes_per_launch"]


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def oracle_rates(run_one, n_items, seconds, threads):
    """Items/s of `run_one(i)` cycling over n_items: one thread, then
    `threads` threads (ctypes releases the GIL inside the oracle)."""
    t0 = time.perf_counter()
    n1 = 0
    while True:
        run_one(n1 % n_items)
        n1 += 1
        if time.perf_counter() - t0 >= seconds:
            break
    single = (n1, time.perf_counter() - t0)
    counts = [0] * threads
    stop = threading.Event()

    def worker(k):
        i = k
        while not stop.is_set():
            run_one(i % n_items)
            counts[k] += 1
            i += threads

    ws = [threading.Thread(target=worker, args=(k,)) for k in range(threads)]
    t1 = time.perf_counter()
    for w in ws:
        w.start()
    time.sleep(seconds)
    stop.set()
    for w in ws:
        w.join()
    multi = (sum(counts), time.perf_counter() - t1)
    return single, multi


def serving_leg(args, torch):
    """Served queries/s at saturation, p50/p99 at 0.5x and 0.9x of it, and the
    same arrival streams served one query at a time with the paper's schedule."""
    from paper_1202_3777_amd.instances import make_serving_trees
    from paper_1202_3777_amd.serve import Clock, Server, TreeExecutor, latency_stats, make_queries
    trees = make_serving_trees(seed=args.seed)
    log(f"[serve] {len(trees)} trees, {sum(t.total_entries() for t in trees):,} entries resident")
    budget = int(args.budget_gib * 2 ** 30)

    def make_exec(capacity, mode, lanes):
        return [TreeExecutor(t, capacity=capacity, mode=mode, lanes=lanes) for t in trees]

    def warm(ex):
        for e in ex:
            e.warm()
        torch.cuda.synchronize()

    def run(ex, rate, n, seed):
        srv = Server(ex, budget_bytes=budget, clock=Clock(torch))
        qs = make_queries(trees, n, rate, seed=seed)
        done = srv.run(qs, max_seconds=240)
        st = latency_stats(done)
        st["batches"] = srv.n_batches
        st["mean_batch"] = float(np.mean(srv.batch_sizes)) if srv.batch_sizes else 0.0
        st["table_bytes"] = int(srv.table_bytes)
        return st

    ex = make_exec(args.capacity, args.serve_mode, args.serve_lanes)
    warm(ex)
    sat = run(ex, None, args.queries, args.seed + 1)
    log(f"[serve] saturated: {sat}")
    lat = {}
    for frac in (0.5, 0.9):
        lat[str(frac)] = run(ex, frac * sat["queries_per_s"], args.queries, args.seed + 2)
        log(f"[serve] rate {frac} x saturated: {lat[str(frac)]}")
    span = sat["n"] / sat["queries_per_s"]
    served_gbs = sat["table_bytes"] / span / 1e9
    del ex
    torch.cuda.empty_cache()
    # the paper's schedule, one query at a time per tree (no batching, one
    # message per launch), on the same arrival streams
    pl = make_exec(1, "plain", 1)
    warm(pl)
    plain_sat = run(pl, None, args.queries // 4, args.seed + 1)
    log(f"[serve] one-query-at-a-time, saturated: {plain_sat}")
    plain_lat = {}
    for frac in (0.5, 0.9):
        plain_lat[str(frac)] = run(pl, frac * sat["queries_per_s"], args.queries // 4, args.seed + 2)
        log(f"[serve] one-query-at-a-time at the batched {frac} x rate: {plain_lat[str(frac)]}")
    del pl
    torch.cuda.empty_cache()
    out = {"workload": "c5: " + WORKLOADS["c5"], "slots_per_tree": args.capacity, "lanes_per_tree": args.serve_lanes,
           "budget_gib": args.budget_gib, "schedule": args.serve_mode, "saturated": sat, "latency": lat,
           "roofline": {"bound": "hbm", "achieved": served_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": served_gbs / HBM_PEAK_GBS,
                        "what": "FP32 table bytes of every served propagation (shared tables once per launch) "
                                "plus the posterior read-out, over the saturated run's wall time"},
           "plain_one_at_a_time": {"saturated": plain_sat, "latency_at_batched_rates": plain_lat}}
    return out, trees


def serving_cpu(args, trees):
    import oracle
    from paper_1202_3777_amd.serve import make_queries
    qs = make_queries(trees, 5000, None, seed=args.seed + 3)
    plans = {i: oracle.Plan.from_instance(trees[i]) for i in range(len(trees))}

    def one(i):
        q = qs[i]
        plans[q.tree].run(trees[q.tree].potentials, q.ev_vars, q.ev_states, want_marginals=False)

    model, avail = host_info()
    threads = max(1, min(16, avail))
    (n1, t1), (nm, tm) = oracle_rates(one, len(qs), args.cpu_seconds, threads)
    return {"value": n1 / t1, "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"{n1} queries of the same mix, FP64, single thread ({t1:.1f} s)",
            "all_core": {"value": nm / tm, "unit": "queries/s", "cores": threads,
                         "sample": f"{nm} queries, {threads} threads ({tm:.1f} s)"},
            "cpu_model": model, "host_cpus_available": avail}


def serve_main(args, torch):
    res, trees = serving_leg(args, torch)
    cpu = None if args.no_cpu_baseline else serving_cpu(args, trees)
    sat = res["saturated"]
    out = {
        "metric": "served queries/s (saturated), with p50/p99 latency at 0.5x and 0.9x of that rate",
        "value": sat["queries_per_s"], "unit": "queries/s", "n_gpus": 1, "steps": args.queries,
        "warmup": args.capacity, "ms_per_step": 1e3 / sat["queries_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded generator, no dataset)",
        "config": {"workload": res["workload"], "seed": args.seed, "slots_per_tree": args.capacity,
                   "lanes_per_tree": args.serve_lanes, "budget_gib": args.budget_gib, "schedule": args.serve_mode,
                   "parallelism": "single GPU"},
        "saturated": sat, "latency": res["latency"], "roofline": res["roofline"],
        "plain_one_at_a_time": res["plain_one_at_a_time"], "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def choose_tuning(args, inst, jt, torch):
    """(tuning, source, candidate table)."""
    from paper_1202_3777_amd import tune
    if args.tuning:
        return json.loads(args.tuning), "given", None
    want = args.autotune == "on" or (args.autotune == "auto" and inst.n_slots > 1)
    if not want:
        return {}, "defaults", None
    key = tune.shape_key(inst, device_name=torch.cuda.get_device_name(0))
    if args.autotune == "auto":
        cached = tune.cache_lookup(key)
        if cached is not None:
            return cached, "cache", None
    log("[bench] autotuning the schedule's shape choices (untimed)")
    tuning, table = tune.autotune(inst, mode=args.mode if args.mode != "plain" else "graph")
    for cand, ms in table:
        log(f"[bench]   {json.dumps(cand):60s} {ms:.4f} ms")
    log(f"[bench] chosen: {json.dumps(tuning)}")
    try:
        tune.cache_store(key, tuning, table, note=f"{inst.name} seed {inst.seed}")
    except OSError:
        pass
    return tuning, "autotuned", table


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
    if args.ceilings:
        ceilings()
        return
    if args.config == "c5":
        serve_main(args, torch)
        return
    log(f"[bench] generating {args.config} seed {args.seed}")
    inst = make_instance(args.config, args.seed)
    tuning, tune_source, tune_table = choose_tuning(args, inst, jt, torch)
    tree = jt.JunctionTree.from_instance(inst, device="cuda:0", tuning=tuning)
    stream = tree.stream
    n_slots = tree.n_slots
    eps = tree.query(jt.JT_Q_ENTRIES_PER_SWEEP)
    entries = 2 * eps * n_slots     # both sweeps, all slots

    def timed(t, mode, steps, warmup):
        for _ in range(warmup):
            t.propagate(mode)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(t.stream)
        for _ in range(steps):
            t.propagate(mode)
        t1.record(t.stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / steps

    log(f"[bench] warmup {args.warmup}, timing {args.steps} steps, mode {args.mode}")
    ms = timed(tree, args.mode, args.steps, args.warmup)
    log(f"[bench] {ms:.4f} ms per propagation")
    bytes_step = tree.query(jt.JT_Q_BYTES_LAST)
    n_launch = tree.query(jt.JT_Q_N_LAUNCHES_PLAIN if args.mode == "plain" else jt.JT_Q_N_LAUNCHES_FUSED)
    shared = tree.query(jt.JT_Q_LAST_SHARED)
    collect_passes = tree.query(jt.JT_Q_LAST_COLLECT_PASSES)
    # every kernel of a propagation is a pass launch (graph replay: the events
    # bracket the launches back to back, so the average launch time here
    # includes the gaps between them and bounds rocprof's kernel time above)
    avg_launch_ms = ms / n_launch
    # algorithmic bytes (every slot computed on its own: per clique and entry
    # 12 B for a leaf, 16 B for an inner clique, 8 B for the root; the unfused
    # schedule's own bytes for the plain mode) and the bytes the executed
    # schedule moved (shared tables counted once per launch)
    alg_step = bytes_step if args.mode == "plain" else tree.query(jt.JT_Q_ALG_BYTES, 0)
    achieved = alg_step / (ms * 1e-3) / 1e9
    executed_gbs = bytes_step / (ms * 1e-3) / 1e9
    copy_gbs = copy_ceiling_gbs(torch)
    log(f"[bench] algorithmic {alg_step / 1e6:.1f} MB per propagation ({achieved:.0f} GB/s); executed schedule "
        f"{bytes_step / 1e6:.1f} MB in {n_launch} launches ({executed_gbs:.0f} GB/s); copy kernel {copy_gbs:.0f} GB/s; "
        f"shared collect {shared}, collect passes {collect_passes}")

    # the paper's schedule, one evidence set at a time
    plain = None
    if not args.no_plain and args.mode != "plain":
        single = jt.JunctionTree(inst.card, inst.clique_off, inst.clique_vars, inst.parent, inst.potentials, 1)
        for s in range(min(2, n_slots)):
            single.set_evidence(0, *inst.evidence[s])
            single.propagate("plain")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(single.stream)
        for s in range(n_slots):
            single.set_evidence(0, *inst.evidence[s])
            single.propagate("plain")
        e1.record(single.stream)
        torch.cuda.synchronize()
        ms_plain = e0.elapsed_time(e1)
        plain = {"ms_per_step": ms_plain, "value": entries / (ms_plain * 1e-3), "unit": "entries/s",
                 "what": f"{n_slots} evidence sets one after the other, each a one-message-at-a-time "
                         f"propagation ({single.query(jt.JT_Q_N_LAUNCHES_PLAIN)} launches per set)",
                 "speedup_of_batched": ms_plain / ms}
        log(f"[bench] one-query-at-a-time sweep: {ms_plain:.3f} ms for {n_slots} sets")
        del single
        tree.propagate(args.mode)
        torch.cuda.synchronize()

    worst = elem = lz_err = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("[bench] oracle: building mapping tables (untimed), checking every slot")
        oplan = oracle.Plan.from_instance(inst)
        worst = elem = lz_err = 0.0
        for s in range(n_slots):
            res = oplan.run(inst.potentials, *inst.evidence[s])
            got, lz = tree.marginals_all(s)
            for c in range(inst.n_cliques):
                a = got[tree.table_off[c]:tree.table_off[c + 1]].astype(np.float64)
                b = oplan.marginal(res, c)
                mb = np.max(np.abs(b))
                worst = max(worst, float(np.max(np.abs(a - b)) / mb))
                big = b >= 1e-3 * mb
                elem = max(elem, float(np.max(np.abs(a[big] - b[big]) / b[big])))
            lz_err = max(lz_err, abs(lz - res["logz"]))
        log(f"[bench] every slot vs FP64: max rel err {worst:.3e}, elementwise {elem:.3e}, |dlogZ| {lz_err:.3e}")

        def one(i):
            oplan.run(inst.potentials, *inst.evidence[i], want_marginals=False)

        model, avail = host_info()
        threads = max(1, min(16, avail))
        (n1, t1), (nm, tm) = oracle_rates(one, n_slots, args.cpu_seconds, threads)
        cpu = {"value": 2 * eps * n1 / t1, "unit": "entries/s", "cores": 1, "kind": "oracle",
               "sample": f"{n1} full FP64 propagations of the same tree, evidence sets cycled ({t1:.1f} s), "
                         "mapping tables prebuilt, single thread",
               "all_core": {"value": 2 * eps * nm / tm, "unit": "entries/s", "cores": threads,
                            "sample": f"{nm} propagations, one evidence set per thread at a time, "
                                      f"{threads} threads ({tm:.1f} s)"},
               "cpu_model": model, "host_cpus_available": avail}
        log(f"[bench] oracle: {t1 / n1:.4f} s per propagation single thread, {tm / nm:.4f} s with {threads} threads")

    serving = None
    if args.config == "c4" and not args.no_serving:
        del tree
        torch.cuda.empty_cache()
        serving, strees = serving_leg(args, torch)
        if not args.no_cpu_baseline:
            serving["cpu_baseline"] = serving_cpu(args, strees)

    value = entries / (ms * 1e-3)
    out = {
        "metric": "BP table entries/s (collect + distribute, sum of |phi_Xi|+|phi_Xk| per message, all evidence sets)",
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
                   "tuning": tuning or "defaults", "tuning_source": tune_source,
                   "autotune_ms": None if tune_table is None else [[c, round(t, 4)] for c, t in tune_table],
                   "shared_collect": bool(shared), "collect_passes": collect_passes,
                   "clique_slot_pairs": inst.n_cliques * n_slots},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.config, "jt_pass", tuning),
                     "kernel": "jt_pass_kernel + jt_pass_multi_kernel (every launch of a propagation)",
                     "launches_per_step": n_launch, "avg_launch_us": avg_launch_ms * 1e3,
                     "bytes": "algorithmic: per clique, slot and table entry 12 B (leaf), 16 B (inner clique), "
                              "8 B (root), FP32 values only" if args.mode != "plain" else
                              "the one-message-at-a-time schedule's FP32 table bytes",
                     "bytes_per_launch": alg_step / n_launch, "bytes_per_step": alg_step,
                     "executed_bytes_per_step": bytes_step, "executed_gbs": executed_gbs,
                     "executed_frac": executed_gbs / HBM_PEAK_GBS,
                     "copy_kernel_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "plain_sweep": plain,
        "max_rel_err_vs_fp64": worst,
        "elem_rel_err_vs_fp64": elem,
        "max_abs_dlogz": lz_err,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
