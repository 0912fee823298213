"""The planner (host C++) under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/plan_check.cpp is compiled with g++ together with the library's
jt_plan.cpp and run on seeded trees: it compiles each plan, builds the
per-propagation schedule of a batched tree for several active-slot counts
and checks every work list, slot set and collect source against an
independent recomputation (see the file's header).  A second build turns
the root-subtree lanes on, so their planning code runs under the sanitizers
too.  CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1202_3777_amd.instances import make_instance, make_serving_trees

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1202_3777_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _build(tmp, defines=()):
    exe = os.path.join(tmp, "plan_check" + "".join(d.split("=")[0] for d in defines))
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"), "-I", CSRC]
                          + [f"-D{d}" for d in defines]
                          + [os.path.join(ROOT, "tests", "plan_check.cpp"), os.path.join(CSRC, "jt_plan.cpp"),
                             "-o", exe])
    return exe


def _write(path, inst, n_slots, target_blocks=0, group_min=0, evidence=None):
    ev = evidence if evidence is not None else [inst.evidence[s % max(1, inst.n_slots)][0] if inst.n_slots else []
                                                for s in range(n_slots)]
    with open(path, "w") as f:
        f.write(f"{inst.n_vars} " + " ".join(map(str, inst.card.tolist())) + "\n")
        f.write(f"{inst.n_cliques} " + " ".join(map(str, inst.clique_off.tolist())) + "\n")
        f.write(f"{inst.clique_vars.shape[0]} " + " ".join(map(str, inst.clique_vars.tolist())) + "\n")
        f.write(" ".join(map(str, inst.parent.tolist())) + "\n")
        f.write(f"{n_slots} {target_blocks} {group_min}\n")
        for s in range(n_slots):
            v = list(map(int, ev[s]))
            f.write(f"{len(v)} " + " ".join(map(str, v)) + "\n")


CASES = [
    ("c4-256", lambda: make_instance("c4", 0), 256, 5120, 0),
    ("c4-12-sparse", lambda: make_instance("c4", 3, n_slots=12, n_obs=(0, 4)), 12, 0, 0),
    ("c4-9-dense", lambda: make_instance("c4", 1, n_slots=9, n_obs=(16, 16)), 9, 1024, 2048),
    ("c1-5", lambda: make_instance("c1", 1, n_slots=5), 5, 0, 0),
    ("c2-3", lambda: make_instance("c2", 2, n_slots=3, n_cliques=12), 3, 0, 0),
    ("c3-1", lambda: make_instance("c3", 1, n_cliques=10), 1, 0, 0),
]


@pytest.fixture(scope="module")
def exes(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("plan_check"))
    return tmp, _build(tmp), _build(tmp, ["JT_LANES_ENABLED=1"])


@pytest.mark.parametrize("name,make,n_slots,tb,gmin", CASES, ids=[c[0] for c in CASES])
def test_planner_schedule_under_sanitizers(exes, name, make, n_slots, tb, gmin):
    tmp, exe, exe_lanes = exes
    inst = make()
    path = os.path.join(tmp, name + ".txt")
    _write(path, inst, n_slots, tb, gmin)
    for e in (exe, exe_lanes):
        r = subprocess.run([e, path], capture_output=True, text=True, timeout=300,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
        print(name, r.stdout.strip(), r.stderr[-2000:])
        assert r.returncode == 0 and r.stdout.startswith("OK"), (name, r.stdout, r.stderr[-2000:])


def test_planner_serving_trees_with_lanes(exes):
    # the serving trees (cardinalities up to 64, separators up to 3 vars) in
    # 4-slot batches, with lanes planned
    tmp, exe, exe_lanes = exes
    rng = np.random.Generator(np.random.PCG64(2))
    for k, inst in enumerate(make_serving_trees(seed=3, n_trees=6, lo=1e3, hi=2e6, max_cliques=20)):
        ev = [rng.choice(inst.n_vars, size=min(3, inst.n_vars), replace=False) for _ in range(4)]
        path = os.path.join(tmp, f"serve{k}.txt")
        _write(path, inst, 4, evidence=ev)
        for e in (exe, exe_lanes):
            r = subprocess.run([e, path], capture_output=True, text=True, timeout=300)
            assert r.returncode == 0 and r.stdout.startswith("OK"), (k, r.stdout, r.stderr[-2000:])
