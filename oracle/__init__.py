"""FP64 CPU oracle for junction-tree belief propagation -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``jt_oracle.c`` (plain C, FP64, sequential
Hugin propagation written from the paper's equations (1)-(3) and Algorithms
1-4) through ctypes and shares nothing with the GPU library.

Pinned by ``tests/test_oracle_*.py``: Fig. 2's printed mapping tables, a
literal quadratic state-string scan, full-joint enumeration, variable
elimination, calibration invariants, the closed form Z = 1 for conditional
tables, and the per-message operation counts of Sec. 3.4.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jt_oracle.c")
_LIB = os.path.join(_HERE, "libjt_oracle.so")

OK = 0
ZERO_EVIDENCE = 1
E_ARG = -1
E_NOT_JT = -2
E_TOO_LARGE = -3
E_NOMEM = -4

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into an in-tree shared library."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f32p = ctypes.POINTER(ctypes.c_float)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.jo_create.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i64p, i32p, i32p, ctypes.POINTER(P)]
    lib.jo_create.restype = ctypes.c_int
    lib.jo_free.argtypes = [P]
    lib.jo_free.restype = None
    lib.jo_mu.argtypes = [P, ctypes.c_int, ctypes.c_int, i32p]
    lib.jo_mu.restype = ctypes.c_int
    lib.jo_map.argtypes = [P, ctypes.c_int, ctypes.c_int, i32p]
    lib.jo_map.restype = ctypes.c_int
    lib.jo_sep_size.argtypes = [P, ctypes.c_int]
    lib.jo_sep_size.restype = ctypes.c_int64
    lib.jo_sep_vars.argtypes = [P, ctypes.c_int, i32p]
    lib.jo_sep_vars.restype = ctypes.c_int
    lib.jo_run.argtypes = [P, f32p, ctypes.c_int, i32p, i32p, f64p, f64p, f64p, i64p]
    lib.jo_run.restype = ctypes.c_int
    lib.jo_mu_scan_literal.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i32p, ctypes.c_int, i32p, i32p]
    lib.jo_mu_scan_literal.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


class Plan:
    """A validated junction tree with separators and mu lists built."""

    def __init__(self, card, clique_off, clique_vars, parent):
        lib = _load()
        self.card = np.ascontiguousarray(card, dtype=np.int32)
        self.clique_off = np.ascontiguousarray(clique_off, dtype=np.int64)
        self.clique_vars = np.ascontiguousarray(clique_vars, dtype=np.int32)
        self.parent = np.ascontiguousarray(parent, dtype=np.int32)
        self.n_cliques = int(self.parent.shape[0])
        h = ctypes.c_void_p()
        rc = lib.jo_create(int(self.card.shape[0]), _ptr(self.card, ctypes.c_int32), self.n_cliques,
                           _ptr(self.clique_off, ctypes.c_int64), _ptr(self.clique_vars, ctypes.c_int32),
                           _ptr(self.parent, ctypes.c_int32), ctypes.byref(h))
        if rc != OK:
            raise OracleError(rc, "jo_create")
        self._h = h
        self._lib = lib
        self.table_size = np.asarray(
            [int(np.prod(self.card[self.clique_vars[self.clique_off[c]:self.clique_off[c + 1]]],
                         dtype=np.int64)) for c in range(self.n_cliques)], dtype=np.int64)
        self.table_off = np.concatenate([[0], np.cumsum(self.table_size)]).astype(np.int64)

    @classmethod
    def from_instance(cls, inst) -> "Plan":
        return cls(inst.card, inst.clique_off, inst.clique_vars, inst.parent)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.jo_free(h)
            self._h = None

    def sep_size(self, child: int) -> int:
        return int(self._lib.jo_sep_size(self._h, child))

    def sep_vars(self, child: int) -> np.ndarray:
        out = np.zeros(64, dtype=np.int32)
        n = self._lib.jo_sep_vars(self._h, child, _ptr(out, ctypes.c_int32))
        if n < 0:
            raise OracleError(n, "jo_sep_vars")
        return out[:n].copy()

    def mu(self, child: int, side: int) -> np.ndarray:
        """mu lists of edge (child, parent(child)) as a [|phi_S|, m] array."""
        c = child if side == 0 else int(self.parent[child])
        out = np.empty(int(self.table_size[c]), dtype=np.int32)
        rc = self._lib.jo_mu(self._h, child, side, _ptr(out, ctypes.c_int32))
        if rc != OK:
            raise OracleError(rc, "jo_mu")
        return out.reshape(self.sep_size(child), -1)

    def csm_map(self, child: int, side: int) -> np.ndarray:
        """Single mapping table: entry r of the clique -> separator index."""
        c = child if side == 0 else int(self.parent[child])
        out = np.empty(int(self.table_size[c]), dtype=np.int32)
        rc = self._lib.jo_map(self._h, child, side, _ptr(out, ctypes.c_int32))
        if rc != OK:
            raise OracleError(rc, "jo_map")
        return out

    def run(self, potentials: np.ndarray, ev_vars: Sequence[int] = (), ev_states: Sequence[int] = (),
            want_marginals: bool = True) -> dict:
        """One full propagation (Algorithm 4) for one evidence set."""
        pot = np.ascontiguousarray(potentials, dtype=np.float32)
        if pot.shape[0] != int(self.table_off[-1]):
            raise ValueError("potentials size mismatch")
        ev = np.ascontiguousarray(ev_vars, dtype=np.int32)
        st = np.ascontiguousarray(ev_states, dtype=np.int32)
        marg = np.empty(int(self.table_off[-1]), dtype=np.float64) if want_marginals else None
        logz = np.zeros(1, dtype=np.float64)
        lzc = np.zeros(self.n_cliques, dtype=np.float64)
        counts = np.zeros(4, dtype=np.int64)
        rc = self._lib.jo_run(self._h, _ptr(pot, ctypes.c_float), int(ev.shape[0]),
                              _ptr(ev, ctypes.c_int32), _ptr(st, ctypes.c_int32),
                              _ptr(marg, ctypes.c_double) if marg is not None else None,
                              _ptr(logz, ctypes.c_double), _ptr(lzc, ctypes.c_double),
                              _ptr(counts, ctypes.c_int64))
        if rc < 0:
            raise OracleError(rc, "jo_run")
        return dict(status=rc, logz=float(logz[0]), logz_per_clique=lzc, marginals=marg,
                    adds=int(counts[0]), muls=int(counts[1]), scale_adds=int(counts[2]),
                    scale_muls=int(counts[3]))

    def marginal(self, res: dict, c: int) -> np.ndarray:
        return res["marginals"][self.table_off[c]:self.table_off[c + 1]]


def mu_scan_literal(card, xvars, svars) -> np.ndarray:
    """The quadratic per-entry state-string scan of Sec. 3.1 (small tables)."""
    lib = _load()
    card = np.ascontiguousarray(card, dtype=np.int32)
    xv = np.ascontiguousarray(xvars, dtype=np.int32)
    sv = np.ascontiguousarray(svars, dtype=np.int32)
    size = int(np.prod(card[xv], dtype=np.int64))
    out = np.empty(size, dtype=np.int32)
    rc = lib.jo_mu_scan_literal(int(card.shape[0]), _ptr(card, ctypes.c_int32), int(xv.shape[0]),
                                _ptr(xv, ctypes.c_int32), int(sv.shape[0]), _ptr(sv, ctypes.c_int32),
                                _ptr(out, ctypes.c_int32))
    if rc != OK:
        raise OracleError(rc, "jo_mu_scan_literal")
    ssize = int(np.prod(card[sv], dtype=np.int64)) if sv.shape[0] else 1
    return out.reshape(ssize, -1)


def run_instance(inst, slot: int = 0, plan: Optional[Plan] = None, want_marginals: bool = True):
    plan = plan or Plan.from_instance(inst)
    ev, st = inst.evidence[slot] if inst.n_slots else (np.zeros(0, np.int32), np.zeros(0, np.int32))
    return plan.run(inst.potentials, ev, st, want_marginals=want_marginals)
