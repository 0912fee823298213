"""Python binding of the junction-tree message engine (``include/jt.h``).

Argument marshalling only: every step of belief propagation runs in the HIP
kernels of ``libjt.so``.  The functions mirror the C ABI one to one;
``JunctionTree`` adds torch-owned device memory and stream handling.  The
binding raises if the built library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjt.so")

JT_OK = 0
JT_E_ARG = -1
JT_E_NOT_JUNCTION_TREE = -2
JT_E_TOO_LARGE = -3
JT_E_NO_MEM = -4
JT_E_HIP = -5
JT_E_ZERO_EVIDENCE = -6
JT_E_STATE = -7

JT_MODE_FUSED = 0
JT_MODE_GRAPH = 1
JT_MODE_PLAIN = 2
JT_MODE_DATAFLOW = 3
JT_MODE_PAPER = 4
JT_MODE_PAPER_GRAPH = 5
MODES = {"fused": JT_MODE_FUSED, "graph": JT_MODE_GRAPH, "plain": JT_MODE_PLAIN, "dataflow": JT_MODE_DATAFLOW,
         "paper": JT_MODE_PAPER, "paper_graph": JT_MODE_PAPER_GRAPH}
JT_LAYOUT_NAIVE = 0
JT_LAYOUT_INTERLEAVED = 1
LAYOUTS = {"naive": JT_LAYOUT_NAIVE, "interleaved": JT_LAYOUT_INTERLEAVED}

JT_Q_N_SLOTS = 0
JT_Q_TOTAL_ENTRIES = 1
JT_Q_TABLE_SIZE = 2
JT_Q_SEP_SIZE = 3
JT_Q_ENTRIES_PER_SWEEP = 4
JT_Q_BYTES_FUSED = 5
JT_Q_BYTES_PLAIN = 6
JT_Q_N_LAUNCHES_FUSED = 7
JT_Q_N_LAUNCHES_PLAIN = 8
JT_Q_HEIGHT = 9
JT_Q_DEPTH = 10
JT_Q_FUSED_LAUNCH_KIND = 11
JT_Q_FUSED_LAUNCH_BYTES = 12
JT_Q_SLOT_BYTES = 13
JT_Q_SHARED_BYTES = 14
JT_Q_ROOT = 15
JT_Q_N_LANES = 16
JT_Q_CLIQUE_LANE = 17
JT_Q_FUSED_LAUNCH_LANE = 18
JT_Q_BYTES_LAST = 19
JT_Q_LAST_SHARED = 20
JT_Q_LAST_COLLECT_PASSES = 21
JT_Q_TOTAL_CLIQUE_VARS = 22
JT_Q_CPT_TOTAL = 23
JT_Q_N_COMPILED_CLIQUES = 24
JT_Q_COMPILED_TABLE_SIZE = 25
JT_Q_LAST_LAUNCH_BYTES = 26
JT_Q_ALG_BYTES = 27
JT_Q_FUSED_LAUNCH_MULTI = 28
JT_Q_FUSED_LAUNCH_BLOCKS = 29

EXPORTED = ["jt_compile_index_maps", "jt_bind", "jt_set_evidence", "jt_propagate", "jt_propagate_n", "jt_marginal",
            "jt_marginals_all", "jt_read_out", "jt_paper_bytes", "jt_paper_bind", "jt_get_index_map", "jt_get_mu_lists", "jt_query", "jt_profile",
            "jt_propagate_scratch", "jt_compile_bn", "jt_bn_structure", "jt_bind_bn", "jt_bn_expected_counts",
            "jt_bn_m_step", "jt_bn_set_cpts", "jt_compile_merged", "jt_free", "jt_last_error"]


class JTError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what} failed with status {code}: {msg}")
        self.code = code


class jt_tuning(ctypes.Structure):
    _fields_ = [("group_min", ctypes.c_int32), ("group_max", ctypes.c_int32), ("group_div", ctypes.c_int32),
                ("target_blocks", ctypes.c_int32), ("max_lanes", ctypes.c_int32), ("task_min", ctypes.c_int32)]


TUNING_FIELDS = [f for f, _ in jt_tuning._fields_]


class jt_bn_desc(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("card", ctypes.POINTER(ctypes.c_int32)),
                ("parent_off", ctypes.POINTER(ctypes.c_int64)), ("parents", ctypes.POINTER(ctypes.c_int32)),
                ("n_slots", ctypes.c_int32), ("tuning", ctypes.POINTER(jt_tuning))]


class jt_tree_desc(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("card", ctypes.POINTER(ctypes.c_int32)),
                ("n_cliques", ctypes.c_int32), ("clique_off", ctypes.POINTER(ctypes.c_int64)),
                ("clique_vars", ctypes.POINTER(ctypes.c_int32)), ("parent", ctypes.POINTER(ctypes.c_int32)),
                ("n_slots", ctypes.c_int32), ("tuning", ctypes.POINTER(jt_tuning))]


_lib = None


def load():
    """Load the in-tree library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1202_3777_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    V, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P32, P64, PF, PD = (ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                        ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double))
    lib.jt_compile_index_maps.argtypes = [ctypes.POINTER(jt_tree_desc), ctypes.POINTER(V), ctypes.POINTER(SZ)]
    lib.jt_bind.argtypes = [V, V, SZ, V, V]
    lib.jt_set_evidence.argtypes = [V, I32, I32, P32, P32]
    lib.jt_propagate.argtypes = [V, I32]
    lib.jt_propagate_n.argtypes = [V, I32, I32]
    lib.jt_marginal.argtypes = [V, I32, I32, V, PD]
    lib.jt_marginals_all.argtypes = [V, I32, V, PD]
    lib.jt_get_index_map.argtypes = [V, I32, I32, P32]
    lib.jt_get_mu_lists.argtypes = [V, I32, I32, P32]
    lib.jt_query.argtypes = [V, I32, I64, P64]
    lib.jt_profile.argtypes = [V, I32, PD, PD, P32, P32]
    lib.jt_propagate_scratch.argtypes = [V, V, V, V, I32, V]
    lib.jt_read_out.argtypes = [V, I32, I32, V, V]
    lib.jt_paper_bytes.argtypes = [V, ctypes.POINTER(SZ)]
    lib.jt_paper_bind.argtypes = [V, V, SZ, I32, I32]
    lib.jt_compile_bn.argtypes = [ctypes.POINTER(jt_bn_desc), ctypes.POINTER(V), ctypes.POINTER(SZ), P32]
    lib.jt_bn_structure.argtypes = [V, P64, P32, P32, P32]
    lib.jt_bind_bn.argtypes = [V, V, SZ, V, V]
    lib.jt_bn_expected_counts.argtypes = [V, I32, V]
    lib.jt_bn_m_step.argtypes = [V, V, ctypes.c_float, V]
    lib.jt_bn_set_cpts.argtypes = [V, V]
    lib.jt_compile_merged.argtypes = [ctypes.POINTER(jt_tree_desc), I32, I64, ctypes.POINTER(V), ctypes.POINTER(SZ),
                                      P32]
    for f in ("jt_compile_index_maps", "jt_bind", "jt_set_evidence", "jt_propagate", "jt_propagate_n", "jt_marginal",
              "jt_marginals_all", "jt_get_index_map", "jt_get_mu_lists", "jt_query", "jt_profile",
              "jt_propagate_scratch", "jt_read_out", "jt_paper_bytes", "jt_paper_bind", "jt_compile_bn",
              "jt_bn_structure", "jt_bind_bn", "jt_bn_expected_counts", "jt_bn_m_step", "jt_bn_set_cpts",
              "jt_compile_merged"):
        getattr(lib, f).restype = I32
    lib.jt_free.argtypes = [V]
    lib.jt_free.restype = None
    lib.jt_last_error.argtypes = []
    lib.jt_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != JT_OK:
        raise JTError(rc, what, load().jt_last_error().decode())


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# --------------------------------------------------------------------------
# one-to-one wrappers of the C ABI

def jt_compile_index_maps(card, clique_off, clique_vars, parent, n_slots: int = 1, tuning: Optional[dict] = None):
    """Returns (handle, device_bytes).  `tuning`: jt_tuning fields by name (missing or 0 = default)."""
    lib = load()
    card = np.ascontiguousarray(card, dtype=np.int32)
    off = np.ascontiguousarray(clique_off, dtype=np.int64)
    cv = np.ascontiguousarray(clique_vars, dtype=np.int32)
    par = np.ascontiguousarray(parent, dtype=np.int32)
    tptr = None
    if tuning:
        unknown = set(tuning) - set(TUNING_FIELDS)
        if unknown:
            raise ValueError(f"unknown tuning fields {sorted(unknown)}")
        tptr = ctypes.pointer(jt_tuning(*[int(tuning.get(f, 0)) for f in TUNING_FIELDS]))
    d = jt_tree_desc(int(card.shape[0]), _p(card, ctypes.c_int32), int(par.shape[0]), _p(off, ctypes.c_int64),
                     _p(cv, ctypes.c_int32), _p(par, ctypes.c_int32), int(n_slots), tptr)
    h = ctypes.c_void_p()
    nbytes = ctypes.c_size_t()
    _check(lib.jt_compile_index_maps(ctypes.byref(d), ctypes.byref(h), ctypes.byref(nbytes)),
           "jt_compile_index_maps")
    return h, int(nbytes.value)


def jt_compile_merged(card, clique_off, clique_vars, parent, max_sep: int, max_entries: int, n_slots: int = 1,
                      tuning: Optional[dict] = None):
    """Returns (handle, device_bytes, n_compiled): the tree with its small
    separators merged away (see include/jt.h)."""
    lib = load()
    card = np.ascontiguousarray(card, dtype=np.int32)
    off = np.ascontiguousarray(clique_off, dtype=np.int64)
    cv = np.ascontiguousarray(clique_vars, dtype=np.int32)
    par = np.ascontiguousarray(parent, dtype=np.int32)
    d = jt_tree_desc(int(card.shape[0]), _p(card, ctypes.c_int32), int(par.shape[0]), _p(off, ctypes.c_int64),
                     _p(cv, ctypes.c_int32), _p(par, ctypes.c_int32), int(n_slots), _tuning_ptr(tuning))
    h = ctypes.c_void_p()
    nbytes = ctypes.c_size_t()
    nm = ctypes.c_int32()
    _check(lib.jt_compile_merged(ctypes.byref(d), int(max_sep), int(max_entries), ctypes.byref(h),
                                 ctypes.byref(nbytes), ctypes.byref(nm)), "jt_compile_merged")
    return h, int(nbytes.value), int(nm.value)


def jt_bind(h, workspace_ptr: int, nbytes: int, init_ptr: int, stream_ptr: int):
    _check(load().jt_bind(h, ctypes.c_void_p(workspace_ptr), nbytes, ctypes.c_void_p(init_ptr),
                          ctypes.c_void_p(stream_ptr)), "jt_bind")


def jt_set_evidence(h, slot: int, vars: Sequence[int], states: Sequence[int]):
    v = np.ascontiguousarray(vars, dtype=np.int32)
    s = np.ascontiguousarray(states, dtype=np.int32)
    if v.shape != s.shape:
        raise ValueError("vars and states differ in length")
    _check(load().jt_set_evidence(h, int(slot), int(v.shape[0]), _p(v, ctypes.c_int32), _p(s, ctypes.c_int32)),
           "jt_set_evidence")


def jt_propagate(h, mode: int = JT_MODE_FUSED):
    _check(load().jt_propagate(h, int(mode)), "jt_propagate")


def jt_propagate_n(h, mode: int, n_active: int):
    _check(load().jt_propagate_n(h, int(mode), int(n_active)), "jt_propagate_n")


def jt_marginal(h, slot: int, clique: int, out_ptr: Optional[int]) -> float:
    lz = ctypes.c_double()
    _check(load().jt_marginal(h, int(slot), int(clique), ctypes.c_void_p(out_ptr or 0), ctypes.byref(lz)),
           "jt_marginal")
    return lz.value


def jt_marginals_all(h, slot: int, out_ptr: Optional[int]) -> float:
    lz = ctypes.c_double()
    _check(load().jt_marginals_all(h, int(slot), ctypes.c_void_p(out_ptr or 0), ctypes.byref(lz)),
           "jt_marginals_all")
    return lz.value


def jt_read_out(h, slot0: int, n: int, posteriors_ptr: int, log_z_ptr: int):
    _check(load().jt_read_out(h, int(slot0), int(n), ctypes.c_void_p(posteriors_ptr), ctypes.c_void_p(log_z_ptr)),
           "jt_read_out")


def _tuning_ptr(tuning):
    if not tuning:
        return None
    unknown = set(tuning) - set(TUNING_FIELDS)
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    return ctypes.pointer(jt_tuning(*[int(tuning.get(f, 0)) for f in TUNING_FIELDS]))


def jt_compile_bn(card, parent_off, parents, n_slots: int = 1, tuning: Optional[dict] = None):
    """Returns (handle, device_bytes, n_cliques)."""
    lib = load()
    card = np.ascontiguousarray(card, dtype=np.int32)
    off = np.ascontiguousarray(parent_off, dtype=np.int64)
    pa = np.ascontiguousarray(parents, dtype=np.int32)
    pa_p = _p(pa, ctypes.c_int32) if pa.shape[0] else ctypes.POINTER(ctypes.c_int32)()
    d = jt_bn_desc(int(card.shape[0]), _p(card, ctypes.c_int32), _p(off, ctypes.c_int64), pa_p, int(n_slots),
                   _tuning_ptr(tuning))
    h = ctypes.c_void_p()
    nbytes = ctypes.c_size_t()
    ncl = ctypes.c_int32()
    _check(lib.jt_compile_bn(ctypes.byref(d), ctypes.byref(h), ctypes.byref(nbytes), ctypes.byref(ncl)),
           "jt_compile_bn")
    return h, int(nbytes.value), int(ncl.value)


def jt_bn_structure(h, n_vars: int, n_cliques: int):
    """(clique_off, clique_vars, parent, family_clique) of a network tree."""
    nvars = jt_query(h, JT_Q_TOTAL_CLIQUE_VARS)
    off = np.empty(n_cliques + 1, dtype=np.int64)
    cv = np.empty(max(1, nvars), dtype=np.int32)
    par = np.empty(n_cliques, dtype=np.int32)
    fam = np.empty(n_vars, dtype=np.int32)
    _check(load().jt_bn_structure(h, _p(off, ctypes.c_int64), _p(cv, ctypes.c_int32), _p(par, ctypes.c_int32),
                                  _p(fam, ctypes.c_int32)), "jt_bn_structure")
    return off, cv[:nvars], par, fam


def jt_bind_bn(h, workspace_ptr: int, nbytes: int, cpts_ptr: int, stream_ptr: int):
    _check(load().jt_bind_bn(h, ctypes.c_void_p(workspace_ptr), nbytes, ctypes.c_void_p(cpts_ptr),
                             ctypes.c_void_p(stream_ptr)), "jt_bind_bn")


def jt_bn_expected_counts(h, n_active: int, counts_ptr: int):
    _check(load().jt_bn_expected_counts(h, int(n_active), ctypes.c_void_p(counts_ptr)), "jt_bn_expected_counts")


def jt_bn_m_step(h, counts_ptr: int, alpha: float, cpts_ptr: int):
    _check(load().jt_bn_m_step(h, ctypes.c_void_p(counts_ptr), float(alpha), ctypes.c_void_p(cpts_ptr)),
           "jt_bn_m_step")


def jt_bn_set_cpts(h, cpts_ptr: int):
    _check(load().jt_bn_set_cpts(h, ctypes.c_void_p(cpts_ptr)), "jt_bn_set_cpts")


def jt_paper_bytes(h) -> int:
    n = ctypes.c_size_t()
    _check(load().jt_paper_bytes(h, ctypes.byref(n)), "jt_paper_bytes")
    return int(n.value)


def jt_paper_bind(h, workspace_ptr: int, nbytes: int, layout: int, threads_per_block: int):
    _check(load().jt_paper_bind(h, ctypes.c_void_p(workspace_ptr), nbytes, int(layout), int(threads_per_block)),
           "jt_paper_bind")


def jt_query(h, what: int, arg: int = 0) -> int:
    out = ctypes.c_int64()
    _check(load().jt_query(h, int(what), int(arg), ctypes.byref(out)), "jt_query")
    return int(out.value)


def jt_get_index_map(h, child: int, side: int, table_size: int) -> np.ndarray:
    out = np.empty(int(table_size), dtype=np.int32)
    _check(load().jt_get_index_map(h, int(child), int(side), _p(out, ctypes.c_int32)), "jt_get_index_map")
    return out


def jt_get_mu_lists(h, child: int, side: int, table_size: int) -> np.ndarray:
    out = np.empty(int(table_size), dtype=np.int32)
    _check(load().jt_get_mu_lists(h, int(child), int(side), _p(out, ctypes.c_int32)), "jt_get_mu_lists")
    return out


def jt_profile(h, mode: int = JT_MODE_FUSED):
    """(pass_ms, finalize_ms, n_pass, n_finalize) of one propagation."""
    pm, fm = ctypes.c_double(), ctypes.c_double()
    npass, nfin = ctypes.c_int32(), ctypes.c_int32()
    _check(load().jt_profile(h, int(mode), ctypes.byref(pm), ctypes.byref(fm), ctypes.byref(npass),
                             ctypes.byref(nfin)), "jt_profile")
    return pm.value, fm.value, npass.value, nfin.value


def jt_propagate_scratch(h, init_ptr: int, posteriors_ptr: int, log_z_ptr: int, mode: int, stream_ptr: int):
    """One propagation of every slot in the library's static device scratch
    (no device allocation); all pointers are device pointers."""
    _check(load().jt_propagate_scratch(h, ctypes.c_void_p(init_ptr), ctypes.c_void_p(posteriors_ptr),
                                       ctypes.c_void_p(log_z_ptr), int(mode), ctypes.c_void_p(stream_ptr)),
           "jt_propagate_scratch")


def jt_free(h):
    if h is not None and h.value:
        load().jt_free(h)


def jt_last_error() -> str:
    return load().jt_last_error().decode()


# --------------------------------------------------------------------------

class JunctionTreePlan:
    """A compiled tree (host side only): index maps and schedule facts."""

    def __init__(self, card, clique_off, clique_vars, parent, n_slots: int = 1, tuning: Optional[dict] = None,
                 merge: Optional[Tuple[int, int]] = None):
        """merge=(max_sep, max_entries): compile with small separators merged
        away (jt_compile_merged); the interface stays the caller's cliques."""
        self.tuning = dict(tuning) if tuning else {}
        self.card = np.ascontiguousarray(card, dtype=np.int32)
        self.clique_off = np.ascontiguousarray(clique_off, dtype=np.int64)
        self.clique_vars = np.ascontiguousarray(clique_vars, dtype=np.int32)
        self.parent = np.ascontiguousarray(parent, dtype=np.int32)
        self.n_cliques = int(self.parent.shape[0])
        self.n_slots = int(n_slots)
        if merge is None:
            self.handle, self.device_bytes = jt_compile_index_maps(self.card, self.clique_off, self.clique_vars,
                                                                   self.parent, n_slots, self.tuning)
        else:
            self.handle, self.device_bytes, self.n_compiled = jt_compile_merged(
                self.card, self.clique_off, self.clique_vars, self.parent, merge[0], merge[1], n_slots, self.tuning)
        self.table_size = np.asarray([jt_query(self.handle, JT_Q_TABLE_SIZE, c) for c in range(self.n_cliques)],
                                     dtype=np.int64)
        self.table_off = np.concatenate([[0], np.cumsum(self.table_size)]).astype(np.int64)

    @classmethod
    def from_instance(cls, inst, n_slots: Optional[int] = None, tuning: Optional[dict] = None, merge=None):
        return cls(inst.card, inst.clique_off, inst.clique_vars, inst.parent,
                   n_slots if n_slots is not None else max(1, inst.n_slots), tuning, merge)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None:
            jt_free(h)
            self.handle = None

    def query(self, what: int, arg: int = 0) -> int:
        return jt_query(self.handle, what, arg)

    def index_map(self, child: int, side: int) -> np.ndarray:
        c = child if side == 0 else int(self.parent[child])
        return jt_get_index_map(self.handle, child, side, int(self.table_size[c]))

    def mu_lists(self, child: int, side: int) -> np.ndarray:
        c = child if side == 0 else int(self.parent[child])
        out = jt_get_mu_lists(self.handle, child, side, int(self.table_size[c]))
        return out.reshape(self.query(JT_Q_SEP_SIZE, child), -1)


class JunctionTree(JunctionTreePlan):
    """A compiled tree bound to torch-owned device memory on one stream."""

    def __init__(self, card, clique_off, clique_vars, parent, potentials: np.ndarray, n_slots: int = 1,
                 device: str = "cuda", stream=None, tuning: Optional[dict] = None, merge=None):
        import torch
        super().__init__(card, clique_off, clique_vars, parent, n_slots, tuning, merge)
        self.torch = torch
        self.device = torch.device(device)
        # a stream of its own: the legacy default stream cannot be captured
        # into a graph (default priority, see the stream rules of the box)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        # allocated on the tree's stream, so that the caching allocator only
        # hands the memory out again after the work queued there (jt_free
        # also waits for that stream before the handle goes)
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(self.device_bytes, dtype=torch.uint8, device=self.device)
        pot = np.ascontiguousarray(potentials, dtype=np.float32)
        if pot.shape[0] != int(self.table_off[-1]):
            raise ValueError("potentials do not match the table sizes")
        init = torch.from_numpy(pot).to(self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        jt_bind(self.handle, self.workspace.data_ptr(), self.device_bytes, init.data_ptr(),
                self.stream.cuda_stream)
        self.stream.synchronize()      # the copy out of `init` is done; it may go
        del init

    @classmethod
    def from_instance(cls, inst, n_slots: Optional[int] = None, **kw):
        t = cls(inst.card, inst.clique_off, inst.clique_vars, inst.parent, inst.potentials,
                n_slots if n_slots is not None else max(1, inst.n_slots), **kw)
        for s, (v, st) in enumerate(inst.evidence[:t.n_slots]):
            t.set_evidence(s, v, st)
        return t

    def set_evidence(self, slot: int, vars: Sequence[int], states: Sequence[int]):
        jt_set_evidence(self.handle, slot, vars, states)

    def propagate(self, mode: str = "fused", n_active: Optional[int] = None):
        if n_active is None:
            jt_propagate(self.handle, MODES[mode])
        else:
            jt_propagate_n(self.handle, MODES[mode], n_active)

    def profile(self, mode: str = "fused"):
        return jt_profile(self.handle, MODES[mode])

    def paper_bind(self, layout: str = "interleaved", threads_per_block: int = 128):
        """Mapping lists for the paper-faithful schedule (modes "paper" and
        "paper_graph"), in a torch-owned workspace of their own."""
        if getattr(self, "paper_workspace", None) is None:
            with self.torch.cuda.stream(self.stream):
                self.paper_workspace = self.torch.empty(jt_paper_bytes(self.handle), dtype=self.torch.uint8,
                                                        device=self.device)
        jt_paper_bind(self.handle, self.paper_workspace.data_ptr(), self.paper_workspace.numel(), LAYOUTS[layout],
                      threads_per_block)

    def marginal(self, slot: int, clique: int) -> Tuple[np.ndarray, float]:
        out = np.empty(int(self.table_size[clique]), dtype=np.float32)
        lz = jt_marginal(self.handle, slot, clique, out.ctypes.data)
        return out, lz

    def marginals_all(self, slot: int):
        out = np.empty(int(self.table_off[-1]), dtype=np.float32)
        lz = jt_marginals_all(self.handle, slot, out.ctypes.data)
        return out, lz

    def marginals_all_device(self, slot: int):
        out = self.torch.empty(int(self.table_off[-1]), dtype=self.torch.float32, device=self.device)
        lz = jt_marginals_all(self.handle, slot, out.data_ptr())
        return out, lz


class BayesNetTree(JunctionTree):
    """A Bayesian network compiled into a junction tree (jt_compile_bn) and
    bound with its conditional tables multiplied into the cliques on the
    device (jt_bind_bn); evidence, propagation and read-out as for any tree,
    plus the EM steps (expected counts, M-step, new tables)."""

    def __init__(self, bn, n_slots: int = 1, device: str = "cuda", stream=None, tuning: Optional[dict] = None):
        import torch
        self.tuning = dict(tuning) if tuning else {}
        self.bn = bn
        self.n_slots = int(n_slots)
        self.handle, self.device_bytes, self.n_cliques = jt_compile_bn(bn.card, bn.parent_off, bn.parents, n_slots,
                                                                       self.tuning)
        self.clique_off, self.clique_vars, self.parent, self.family_clique = jt_bn_structure(
            self.handle, bn.n_vars, self.n_cliques)
        self.card = np.ascontiguousarray(bn.card, dtype=np.int32)
        self.table_size = np.asarray([jt_query(self.handle, JT_Q_TABLE_SIZE, c) for c in range(self.n_cliques)],
                                     dtype=np.int64)
        self.table_off = np.concatenate([[0], np.cumsum(self.table_size)]).astype(np.int64)
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(self.device_bytes, dtype=torch.uint8, device=self.device)
            self.cpts = torch.from_numpy(np.ascontiguousarray(bn.cpts, dtype=np.float32)).to(self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        jt_bind_bn(self.handle, self.workspace.data_ptr(), self.device_bytes, self.cpts.data_ptr(),
                   self.stream.cuda_stream)

    def clique_vars_of(self, c: int) -> np.ndarray:
        return self.clique_vars[self.clique_off[c]:self.clique_off[c + 1]]

    def expected_counts(self, n_active: Optional[int] = None):
        """Device tensor of sum over slots of P(family | e_slot), laid out like the tables."""
        with self.torch.cuda.stream(self.stream):
            out = self.torch.empty(int(jt_query(self.handle, JT_Q_CPT_TOTAL)), dtype=self.torch.float32,
                                   device=self.device)
        jt_bn_expected_counts(self.handle, n_active or self.n_slots, out.data_ptr())
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)   # later torch work sees the result
        return out

    def m_step(self, counts, alpha: float = 0.0):
        with self.torch.cuda.stream(self.stream):
            out = self.torch.empty_like(counts)
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        jt_bn_m_step(self.handle, counts.data_ptr(), alpha, out.data_ptr())
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def set_cpts(self, cpts):
        """New conditional tables (device tensor): the clique tables are
        recomputed on the device before the next propagation."""
        self.cpts = cpts
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        jt_bn_set_cpts(self.handle, cpts.data_ptr())
