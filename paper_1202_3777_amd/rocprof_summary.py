"""Summaries of rocprofv3 output for the engine's kernels.

    python -m paper_1202_3777_amd.rocprof_summary stats DIR
        per-kernel calls / average / total from a --kernel-trace --stats run
    python -m paper_1202_3777_amd.rocprof_summary launches DIR --config CFG [--tuning JSON]
        launch by launch of the last propagation in a --kernel-trace run of
        bench.py: kernel, grid, start, duration, the FP32 table bytes the
        launch moved and the bytes / duration rate.  The bytes come from the
        library itself (one propagation of the same seeded workload, then
        jt_query(JT_Q_LAST_LAUNCH_BYTES)), so this step needs the GPU.
    python -m paper_1202_3777_amd.rocprof_summary traffic --kernel PREFIX \
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --copy-bytes N \
        --out FILE.json
        HBM bytes per launch of the kernels whose names start with PREFIX
        (all dispatches of all of them averaged: the propagation's pass
        kernels) from two counter runs (FETCH_SIZE, then WRITE_SIZE), each
        scaled by what the same counter reads for a plain copy of N bytes
        (the runtime's copy kernel) so that the counter's unit and coverage
        are calibrated on this GPU.

    python -m paper_1202_3777_amd.rocprof_summary counters DIR... --launches N
        per launch of the last propagation (the last N dispatches of the pass
        kernels) the SQ / TCP counters of one or more --pmc runs of the same
        command: waves, cycles per wave, the share of wave cycles spent
        waiting and issuing VALU instructions, instructions per wave, the
        mean L2 read and write latency seen from the L1 (cycles).

The traffic file records the sha256 of the kernel source it was measured
on; bench.py reports the traffic only while the source is unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "jt_kernels.hip")


PLAN_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("jt_plan.cpp", "jt_plan.h", "jt_internal.h")]


def kernel_source_hash() -> str:
    return hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()


def plan_source_hash() -> str:
    """sha256 over the planner's sources: the schedule (launches, groups,
    work lists) that the kernels run, and so the bytes they move."""
    h = hashlib.sha256()
    for f in PLAN_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def _csv(d, pattern):
    files = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not files:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return list(csv.DictReader(open(sorted(files)[0])))


def counter_per_dispatch(d, counter):
    """{kernel name: [value per dispatch]} from a --pmc run."""
    rows = _csv(d, "*counter_collection.csv")
    acc = defaultdict(lambda: defaultdict(float))
    for r in rows:
        if r.get("Counter_Name", "") != counter:
            continue
        name = r.get("Kernel_Name", "")
        did = r.get("Dispatch_Id", r.get("Correlation_Id", "0"))
        acc[name][did] += float(r["Counter_Value"])
    return {k: [v[x] for x in sorted(v, key=lambda s: int(s))] for k, v in acc.items()}


def stats(d):
    rows = _csv(d, "*kernel_stats.csv")
    return [{"name": r["Name"], "calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
             "total_ns": int(float(r["TotalDurationNs"])), "pct": float(r["Percentage"])} for r in rows]


def launches(d, config, tuning=None, seed=0, kernel="jt_pass"):
    """Rows of the last propagation's launches: (kernel, grid blocks, start us, dur us, bytes)."""
    from paper_1202_3777_amd import jt
    from paper_1202_3777_amd.instances import make_instance
    rows = [r for r in _csv(d, "*kernel_trace.csv") if r["Kernel_Name"].startswith(kernel)]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    inst = make_instance(config, seed)
    tree = jt.JunctionTree.from_instance(inst, device="cuda:0", tuning=tuning)
    tree.propagate("fused")
    n = tree.query(jt.JT_Q_N_LAUNCHES_FUSED)
    last = rows[-n:]
    t0 = int(last[0]["Start_Timestamp"])
    # a level's multi-slot launch runs beside its one-slot launch, so the two
    # may start in either order: match trace rows to launches by kernel
    multi = [tree.query(jt.JT_Q_FUSED_LAUNCH_MULTI, i) for i in range(n)]
    byname = {True: [r for r in last if "multi" in r["Kernel_Name"]],
              False: [r for r in last if "multi" not in r["Kernel_Name"]]}
    used = {True: 0, False: 0}
    out = []
    for i in range(n):
        m = bool(multi[i])
        r = byname[m][used[m]]
        used[m] += 1
        s, e = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        grid = int(r.get("Grid_Size_X", r.get("Grid_Size", 0))) // int(r.get("Workgroup_Size_X", 256) or 256)
        name = r["Kernel_Name"].split("(")[0]
        out.append((name, grid, (s - t0) / 1e3, (e - s) / 1e3, tree.query(jt.JT_Q_LAST_LAUNCH_BYTES, i)))
    span = (max(int(r["End_Timestamp"]) for r in last) - t0) / 1e3
    return out, span


def _match(d, prefix):
    """Values of every dispatch of the kernels whose names start with prefix."""
    names = sorted(k for k in d if k.startswith(prefix))
    if not names:
        raise KeyError(f"no kernel {prefix}* in counter output ({list(d)[:5]})")
    return names, [x for k in names for x in d[k]]


def traffic(args):
    names, fetch = _match(counter_per_dispatch(args.fetch, "FETCH_SIZE"), args.kernel)
    _, write = _match(counter_per_dispatch(args.write, "WRITE_SIZE"), args.kernel)
    cf = counter_per_dispatch(args.copy_fetch, "FETCH_SIZE")
    cw = counter_per_dispatch(args.copy_write, "WRITE_SIZE")
    # the reference copy kernel (torch's device-to-device copy); other
    # kernels in that run (e.g. the fill that initializes the source) are not it
    cfk = next(k for k in cf if "copyBuffer" in k or "copy" in k.lower())
    cwk = next(k for k in cw if "copyBuffer" in k or "copy" in k.lower())
    cfv = sorted(cf[cfk])[len(cf[cfk]) // 2]
    cwv = sorted(cw[cwk])[len(cw[cwk]) // 2]
    f_scale = args.copy_bytes / cfv          # bytes per counter unit, reads
    w_scale = args.copy_bytes / cwv          # bytes per counter unit, writes
    fb = sum(fetch) / len(fetch) * f_scale
    wb = sum(write) / len(write) * w_scale
    out = {"kernel": args.kernel, "kernels": [k.split("(")[0] for k in names],
           "source_sha256": kernel_source_hash(),
           "plan_sha256": plan_source_hash(),
           "dispatches": [len(fetch), len(write)],
           "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "traffic_bytes_per_launch": fb + wb,
           "copy_kernel": [cfk, cwk], "copy_bytes": args.copy_bytes,
           "copy_counter_fetch": cfv, "copy_counter_write": cwv,
           "scale_bytes_per_unit": [f_scale, w_scale], "workload": args.workload,
           "tuning": json.loads(args.tuning) if args.tuning else {}}
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def counters(dirs, n_launch, kernel="jt_pass"):
    """{launch index: {counter: value}} over the last n_launch pass dispatches."""
    per = defaultdict(dict)
    for d in dirs:
        disp = defaultdict(dict)
        for r in _csv(d, "*counter_collection.csv"):
            if not r["Kernel_Name"].startswith(kernel):
                continue
            did = int(r["Dispatch_Id"])
            disp[did][r["Counter_Name"]] = disp[did].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            disp[did]["_kernel"] = r["Kernel_Name"].split("(")[0]
        for i, did in enumerate(sorted(disp)[-n_launch:]):
            per[i].update(disp[did])
    return per


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    l = sub.add_parser("launches")
    l.add_argument("dir")
    l.add_argument("--config", required=True)
    l.add_argument("--tuning", default=None)
    l.add_argument("--seed", type=int, default=0)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--workload", default="")
    t.add_argument("--tuning", default=None, help="JSON of the shape choices the counter runs used")
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--launches", type=int, required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        for r in stats(a.dir):
            print(f"{r['name'][:40]:40s} calls {r['calls']:6d} avg {r['avg_ns'] / 1e3:9.2f} us "
                  f"total {r['total_ns'] / 1e6:9.3f} ms {r['pct']:6.2f} %")
    elif a.cmd == "launches":
        rows, span = launches(a.dir, a.config, json.loads(a.tuning) if a.tuning else None, a.seed)
        busy = 0.0
        for i, (name, g, st, du, b) in enumerate(rows):
            busy += du
            print(f"{i:3d} {name:22s} grid {g:7d} blk start {st:8.1f} dur {du:8.1f} us "
                  f"{b / 2**20:9.1f} MiB {b / (du * 1e3):7.0f} GB/s")
        print(f"span {span:.1f} us, kernels busy {busy:.1f} us (launches of one level overlap)")
    elif a.cmd == "counters":
        per = counters(a.dirs, a.launches)
        print(f"{'#':>3} {'kernel':22s} {'waves':>6} {'cyc/wave':>8} {'wait%':>6} {'valu%':>6} {'valu/w':>7} "
              f"{'salu/w':>7} {'vmem/w':>7} {'lds/w':>6} {'rd lat':>7} {'wr lat':>7}")
        for i in sorted(per):
            x = per[i]
            w = max(1.0, x.get("SQ_WAVES", 1.0))
            wc = max(1.0, x.get("SQ_WAVE_CYCLES", 1.0))
            rl = x.get("TCP_TCC_READ_REQ_LATENCY_sum", 0.0) / max(1.0, x.get("TCP_TCC_READ_REQ_sum", 1.0))
            wl = x.get("TCP_TCC_WRITE_REQ_LATENCY_sum", 0.0) / max(1.0, x.get("TCP_TCC_WRITE_REQ_sum", 1.0))
            print(f"{i:3d} {x.get('_kernel', '')[:22]:22s} {w:6.0f} {wc / w:8.0f} {100 * x.get('SQ_WAIT_ANY', 0) / wc:6.1f} "
                  f"{100 * x.get('SQ_ACTIVE_INST_VALU', 0) / wc:6.1f} {x.get('SQ_INSTS_VALU', 0) / w:7.0f} "
                  f"{x.get('SQ_INSTS_SALU', 0) / w:7.0f} {x.get('SQ_INSTS_VMEM', 0) / w:7.0f} "
                  f"{x.get('SQ_INSTS_LDS', 0) / w:6.0f} {rl:7.0f} {wl:7.0f}")
    else:
        traffic(a)


if __name__ == "__main__":
    sys.exit(main())
