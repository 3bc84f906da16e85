"""The paper's multi-core CPU variant of RAKS (Section 4.2.4 "Scheduling":
OpenMP, a thread per frontier for all its keywords, dynamic scheduling), as a
host baseline beside the GPU library.  Built from ``raks_cpu.c`` with gcc.

It is not a fallback of the GPU path and shares no code with it or with the
reference implementation; its results and counters equal the reference's.
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libraks_cpu.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, os.path.join(_HERE, "raks_cpu.c"), "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("A", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("label", ctypes.c_void_p), ("vocab", ctypes.c_int32),
                ("kw_ptr", ctypes.c_void_p), ("kw_nodes", ctypes.c_void_p)]


class _Query(ctypes.Structure):
    _fields_ = [("central", ctypes.c_void_p), ("n_central", ctypes.c_int32),
                ("marginal", ctypes.c_void_p), ("n_marginal", ctypes.c_int32),
                ("k", ctypes.c_int32), ("w", ctypes.c_int32), ("gamma_num", ctypes.c_int32),
                ("gamma_den", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("score_mode", ctypes.c_int32), ("rerank", ctypes.c_int32)]


@functools.lru_cache(maxsize=1)
def _lib():
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    lib.rcpu_query.argtypes = [ctypes.POINTER(_Graph), ctypes.c_void_p, ctypes.POINTER(_Query),
                               ctypes.c_int, ctypes.POINTER(ctypes.POINTER(ctypes.c_int64)),
                               ctypes.POINTER(ctypes.c_int64)]
    lib.rcpu_free.argtypes = [ctypes.c_void_p]
    lib.rcpu_activation.argtypes = [ctypes.POINTER(_Graph), ctypes.c_void_p, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.rcpu_explore.argtypes = [ctypes.POINTER(_Graph), ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                 ctypes.c_void_p]
    return lib


_END = {0: "none", 1: "exhausted", 2: "stop", 3: "level_bound", 4: "empty_keyword"}
_STATS = ("levels", "end_reason", "frontier", "e_arc", "e_alg", "gate_pass", "h_writes")


def _decode(w) -> dict:
    """The int64 result words (same layout as the reference's) as a dict."""
    w = [int(x) for x in w]
    stats = []
    for s in range(2):
        d = dict(zip(_STATS, w[3 + 7 * s: 10 + 7 * s]))
        d["end"] = _END.get(d["end_reason"], "?")
        stats.append(d)
    out = {"status": w[0], "n_cg": w[2], "stats": stats, "results": []}
    p = 17
    for _ in range(w[1]):
        central, sc, sm, key, wsum, nn = w[p:p + 6]
        p += 6
        nodes = tuple(w[p:p + nn])
        p += nn
        na = w[p]
        p += 1
        arcs = tuple((w[p + 3 * i], w[p + 3 * i + 1], w[p + 3 * i + 2]) for i in range(na))
        p += 3 * na
        out["results"].append({"central": central, "score_c": sc, "score_m": sm, "key": key,
                               "weight_sum": wsum, "nodes": nodes, "arcs": arcs})
    return out


class CpuRaks:
    """One graph; queries run on ``threads`` host threads (0 = all)."""

    def __init__(self, g):
        self._arrs = [np.ascontiguousarray(g.row_ptr, np.int64), np.ascontiguousarray(g.col, np.int32),
                      np.ascontiguousarray(g.label, np.uint16), np.ascontiguousarray(g.kw_ptr, np.int64),
                      np.ascontiguousarray(g.kw_nodes, np.int32)]
        rp, col, lab, kp, kn = self._arrs
        self._nw = np.ascontiguousarray(g.node_weight, np.uint8)
        self._g = _Graph(int(g.n_nodes), int(col.shape[0]), rp.ctypes.data, col.ctypes.data,
                         lab.ctypes.data, int(kp.shape[0] - 1), kp.ctypes.data, kn.ctypes.data)

    def activation(self, abar: float, alpha: float, mode: int = 0, threads: int = 0):
        """Per-arc activation levels (uint8 [A]) computed by this variant on
        ``threads`` host threads (0 = all); mode 0 per arc, 1 per node."""
        act = np.empty(self._arrs[1].shape[0], np.uint8)
        rc = _lib().rcpu_activation(ctypes.byref(self._g), self._nw.ctypes.data, float(abar),
                                    float(alpha), int(mode), int(threads), act.ctypes.data)
        if rc != 0:
            raise ValueError(f"activation failed ({rc})")
        return act

    def explore(self, act, keywords, block: bool = False, max_level: int = 20,
                threads: int = 0) -> dict:
        """Exploration alone (Algorithm 1) from the keywords' node sets; its counters."""
        act = np.ascontiguousarray(act, np.uint8)
        kws = np.ascontiguousarray(keywords, np.int32)
        out = np.zeros(7, np.int64)
        rc = _lib().rcpu_explore(ctypes.byref(self._g), act.ctypes.data, kws.ctypes.data,
                                 int(kws.shape[0]), int(bool(block)), int(max_level), int(threads),
                                 out.ctypes.data)
        if rc != 0:
            raise ValueError(f"exploration failed ({rc})")
        d = {k: int(v) for k, v in zip(_STATS, out)}
        d["end"] = _END.get(d["end_reason"], "?")
        return d

    def query(self, act, q, threads: int = 0) -> dict:
        act = np.ascontiguousarray(act, np.uint8)
        c = np.ascontiguousarray(q.central, np.int32)
        m = np.ascontiguousarray(q.marginal if len(q.marginal) else [0], np.int32)
        cq = _Query(c.ctypes.data, len(q.central), m.ctypes.data, len(q.marginal), q.k, q.w,
                    q.gamma_num, q.gamma_den, q.max_level, getattr(q, "score_mode", 0),
                    getattr(q, "rerank", 0))
        buf = ctypes.POINTER(ctypes.c_int64)()
        ln = ctypes.c_int64(0)
        rc = _lib().rcpu_query(ctypes.byref(self._g), act.ctypes.data, ctypes.byref(cq),
                               int(threads), ctypes.byref(buf), ctypes.byref(ln))
        if rc != 0:
            raise ValueError(f"query failed ({rc})")
        try:
            words = np.ctypeslib.as_array(buf, shape=(ln.value,)).copy()
        finally:
            _lib().rcpu_free(buf)
        return _decode(words)
