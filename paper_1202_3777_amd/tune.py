"""Autotuner for the shape choices of the fused schedule.

The tile of a clique is fixed by its table layout (the innermost
cardinalities); what can be chosen per tree is how the work is cut: the size
of a group (the entries one block reduces into one partial row), the blocks a
launch aims for, and how many streams the root's subtrees are spread over
(`jt_tuning` in include/jt.h).  The tuner compiles the tree once per
candidate, times propagations of the same evidence on the GPU and keeps the
fastest.  Every candidate computes the same messages; results differ only by
rounding order and stay within the stated tolerance.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Callable, Dict, List, Optional, Sequence, Tuple

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
KERNEL_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "jt_kernels.hip")
PLAN_SOURCES = [os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f)
                for f in ("jt_plan.cpp", "jt_plan.h", "jt_internal.h")]

# Candidates around the built-in defaults (group 8K..32K entries, 1280 blocks
# per launch): one knob moved at a time, joint moves, and smaller least work
# per block (task_min) at several block targets.  (Lanes are
# disabled in the library, so max_lanes is not searched.)
DEFAULT_CANDIDATES: List[Dict[str, int]] = [
    {},
    {"group_min": 2048},
    {"group_min": 4096},
    {"group_min": 16384},
    {"group_div": 512},
    {"group_div": 2048},
    {"target_blocks": 1024},
    {"target_blocks": 2560},
    {"target_blocks": 5120},
    {"target_blocks": 10240},
    {"target_blocks": 20480},
    {"group_min": 16384, "target_blocks": 2560},
    {"group_min": 4096, "target_blocks": 1024},
    {"group_min": 2048, "group_div": 512},
    {"task_min": 1},
    {"task_min": 1, "target_blocks": 5120},
    {"task_min": 1, "target_blocks": 10240},
    {"task_min": 1, "target_blocks": 20480},
    {"task_min": 2048, "target_blocks": 10240},
    {"task_min": 2048, "target_blocks": 20480},
]


def choose(candidates: Sequence[Dict[str, int]], timer: Callable[[Dict[str, int]], float],
           finalists: int = 3, rounds: int = 3) -> Tuple[Dict[str, int], List[Tuple[Dict[str, int], float]]]:
    """Time every candidate once with `timer` (ms per propagation), then time
    the `finalists` fastest again, taking turns, `rounds` more times each, and
    return the candidate with the lowest time seen (the earliest listed among
    equals) with the table of every candidate's lowest time.  One timing of a
    launch-bound schedule can be off by a percent or two, as much as the gaps
    between the leading candidates; alternating repeats separate them."""
    table = [[dict(c), float(timer(c))] for c in candidates]
    top = sorted(range(len(table)), key=lambda i: (table[i][1], i))[:max(0, finalists)]
    for _ in range(rounds):
        for i in top:
            table[i][1] = min(table[i][1], float(timer(table[i][0])))
    best = min(range(len(table)), key=lambda i: (table[i][1], i))
    return table[best][0], [(c, t) for c, t in table]


def gpu_timer(inst, n_slots: Optional[int] = None, mode: str = "graph", steps: int = 10, warmup: int = 2,
              device: str = "cuda:0") -> Callable[[Dict[str, int]], float]:
    """ms per propagation of `inst` (its own evidence) for one candidate."""
    import torch

    from paper_1202_3777_amd import jt

    def run(cand: Dict[str, int]) -> float:
        tree = jt.JunctionTree.from_instance(inst, n_slots=n_slots, device=device, tuning=cand)
        for _ in range(warmup):
            tree.propagate(mode)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(tree.stream)
        for _ in range(steps):
            tree.propagate(mode)
        b.record(tree.stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        del tree
        torch.cuda.empty_cache()
        return ms

    return run


def autotune(inst, n_slots: Optional[int] = None, candidates: Optional[Sequence[Dict[str, int]]] = None,
             **timer_kw) -> Tuple[Dict[str, int], List[Tuple[Dict[str, int], float]]]:
    """Pick the fastest shape choice for `inst` on the GPU."""
    return choose(candidates if candidates is not None else DEFAULT_CANDIDATES,
                  gpu_timer(inst, n_slots=n_slots, **timer_kw))


def shape_key(inst, n_slots: Optional[int] = None, device_name: str = "") -> str:
    """Shape class of a tree for the tuning cache: what the shape choices
    depend on -- the tree's topology, every table and separator size, the
    table layouts (tiles), the slot count, the GPU, the pass kernels' source
    and the planner's (which lays out the launches the choices cut) -- and
    nothing of the potentials or the evidence."""
    h = hashlib.sha256()
    for f in [KERNEL_SOURCE] + PLAN_SOURCES:
        h.update(open(f, "rb").read())
    for a in (inst.card, inst.clique_off, inst.clique_vars, inst.parent):
        h.update(a.tobytes())
    h.update(str(int(n_slots if n_slots is not None else max(1, inst.n_slots))).encode())
    h.update(device_name.encode())
    return h.hexdigest()[:32]


def cache_lookup(key: str, path: str = CACHE_PATH) -> Optional[Dict[str, int]]:
    if not os.path.exists(path):
        return None
    try:
        entry = json.load(open(path)).get(key)
    except (OSError, ValueError):
        return None
    return None if entry is None else dict(entry["tuning"])


def cache_store(key: str, tuning: Dict[str, int], table, note: str = "", path: str = CACHE_PATH) -> None:
    data = {}
    if os.path.exists(path):
        try:
            data = json.load(open(path))
        except ValueError:
            data = {}
    data[key] = {"tuning": dict(tuning), "note": note,
                 "candidates_ms": [[c, round(ms, 4)] for c, ms in table]}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
