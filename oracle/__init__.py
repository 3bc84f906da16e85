"""Reference implementation of RAKS (test infrastructure only).

Plain single-threaded C (``raks_oracle.c``) behind ctypes.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import this
package; the GPU library never does, and the two share no code.

Parity status per function (what pins it is in ``tests/test_oracle_pins.py``):
  activation        pinned (Theorem 1 bounds, exact special values)
  explore           pinned (brute-force path scores, Dial-bucket label setting,
                    plain BFS special cases, order-independence)
  query / run 1     pinned (identification vs. brute force, recovery vs.
                    brute-force prefix-optimal paths, invariants)
  query / run 2     pinned in part (S^m and keys vs. the Dial formulation;
                    marginal recovery vs. brute force for one marginal keyword
                    and vs. path enumeration of the blocked H for two and
                    three; Theorem 4 vs. a run without early termination);
                    the PTC guard, the tie-breaks and gamma follow stated
                    readings and are otherwise parity unpinned.
  work counters     pinned (tests/test_oracle_counters.py: frontier sizes,
  and status bits   e_arc, e_alg, gate_pass, h_writes and the level-bound
                    bits derived from Dial distances and Algorithm 1's
                    frontier rule, plus hand-counted graphs)
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

MODE_EDGE, MODE_NODE = 0, 1
FLAG_NO_CG_BLOCK, FLAG_NO_THM4, FLAG_NO_M_BLOCK = 1, 2, 4
END_NAMES = {0: "none", 1: "exhausted", 2: "stop", 3: "level_bound", 4: "empty_keyword"}


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-o", tmp,
                               os.path.join(_HERE, "raks_oracle.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("A", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("label", ctypes.c_void_p),
                ("node_weight", ctypes.c_void_p), ("vocab", ctypes.c_int32),
                ("kw_ptr", ctypes.c_void_p), ("kw_nodes", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in
                ("levels", "end_reason", "frontier", "e_arc", "e_alg", "gate_pass", "h_writes")]


class _Query(ctypes.Structure):
    _fields_ = [("central", ctypes.c_void_p), ("n_central", ctypes.c_int32),
                ("marginal", ctypes.c_void_p), ("n_marginal", ctypes.c_int32),
                ("k", ctypes.c_int32), ("w", ctypes.c_int32), ("gamma_num", ctypes.c_int32),
                ("gamma_den", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("score_mode", ctypes.c_int32), ("rerank", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("shuffle", ctypes.c_uint64)]


@functools.lru_cache(maxsize=1)
def _lib():
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_check_graph.argtypes = [ctypes.POINTER(_Graph)]
    lib.orc_level_of.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.orc_activation.argtypes = [ctypes.POINTER(_Graph), ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]
    lib.orc_explore.argtypes = [ctypes.POINTER(_Graph), ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                ctypes.c_void_p, ctypes.POINTER(_Stats)]
    lib.orc_query.argtypes = [ctypes.POINTER(_Graph), ctypes.c_void_p, ctypes.POINTER(_Query),
                              ctypes.POINTER(ctypes.POINTER(ctypes.c_int64)),
                              ctypes.POINTER(ctypes.c_int64)]
    lib.orc_free.argtypes = [ctypes.c_void_p]
    return lib


def level_of(x: float, abar: float, alpha: float) -> int:
    """Eqs. 1-3 for one rescaled weight x."""
    return int(_lib().orc_level_of(x, abar, alpha))


def _stats_dict(vals):
    keys = ("levels", "end_reason", "frontier", "e_arc", "e_alg", "gate_pass", "h_writes")
    d = {k: int(v) for k, v in zip(keys, vals)}
    d["end"] = END_NAMES.get(d["end_reason"], "?")
    return d


class Oracle:
    """Reference search over one graph (arrays from ``synth.Graph`` or alike)."""

    def __init__(self, g, check: bool = True):
        self.g = g
        self._keep = [np.ascontiguousarray(a) for a in
                      (g.row_ptr, g.col, g.label, g.node_weight, g.kw_ptr, g.kw_nodes)]
        rp, col, lab, nw, kp, kn = self._keep
        self._cg = _Graph(int(g.n_nodes), int(col.shape[0]), rp.ctypes.data, col.ctypes.data,
                          lab.ctypes.data, nw.ctypes.data, int(kp.shape[0] - 1),
                          kp.ctypes.data, kn.ctypes.data)
        if check:
            rc = _lib().orc_check_graph(ctypes.byref(self._cg))
            if rc != 0:
                raise ValueError(f"graph violates the input contract (code {rc})")

    def activation(self, abar: float, alpha: float, mode: int = MODE_EDGE, want_x: bool = False):
        """Per-arc activation levels (uint8 [A]); NODE mode also returns the
        per-node levels.  With ``want_x`` the rescaled weights (and, in EDGE
        mode, the label counts c) come back too."""
        A, n = int(self._cg.A), int(self._cg.n)
        act = np.empty(A, np.uint8)
        act_node = np.empty(n, np.uint8) if mode == MODE_NODE else None
        x = np.empty(A if mode == MODE_EDGE else n, np.float64) if want_x else None
        c = np.empty(A, np.int64) if (want_x and mode == MODE_EDGE) else None
        rc = _lib().orc_activation(ctypes.byref(self._cg), abar, alpha, mode, act.ctypes.data,
                                   act_node.ctypes.data if act_node is not None else None,
                                   x.ctypes.data if x is not None else None,
                                   c.ctypes.data if c is not None else None)
        if rc != 0:
            raise ValueError(f"activation failed ({rc})")
        if want_x:
            return act, act_node, x, c
        return (act, act_node) if mode == MODE_NODE else act

    def explore(self, act, keywords, block: bool = False, max_level: int = 20, shuffle: int = 0):
        """Algorithm 1 run to exhaustion or the level bound, with no result
        identification.  Returns (H [n x T] uint8, stats dict)."""
        act = np.ascontiguousarray(act, np.uint8)
        kws = np.ascontiguousarray(keywords, np.int32)
        T = int(kws.shape[0])
        H = np.empty((int(self._cg.n), T), np.uint8)
        st = _Stats()
        rc = _lib().orc_explore(ctypes.byref(self._cg), act.ctypes.data, kws.ctypes.data, T,
                                int(block), max_level, shuffle, H.ctypes.data, ctypes.byref(st))
        if rc != 0:
            raise ValueError(f"explore failed ({rc})")
        return H, _stats_dict([getattr(st, f) for f, _ in _Stats._fields_])

    def query(self, act, q, flags: int = 0, shuffle: int = 0, lean: bool = False) -> dict:
        """Both runs, recovery and ranking for one radial pattern query.  With
        ``lean`` the node and arc lists come back as int32 numpy arrays (for
        results of hundreds of millions of arcs)."""
        act = np.ascontiguousarray(act, np.uint8)
        c = np.ascontiguousarray(q.central, np.int32)
        m = np.ascontiguousarray(q.marginal if len(q.marginal) else [0], np.int32)
        cq = _Query(c.ctypes.data, len(q.central), m.ctypes.data, len(q.marginal), q.k,
                    q.w, q.gamma_num, q.gamma_den, q.max_level, getattr(q, "score_mode", 0),
                    getattr(q, "rerank", 0), flags, shuffle)
        buf = ctypes.POINTER(ctypes.c_int64)()
        ln = ctypes.c_int64(0)
        rc = _lib().orc_query(ctypes.byref(self._cg), act.ctypes.data, ctypes.byref(cq),
                              ctypes.byref(buf), ctypes.byref(ln))
        if rc != 0:
            raise ValueError(f"query failed ({rc})")
        try:
            words = np.ctypeslib.as_array(buf, shape=(ln.value,)).copy()
        finally:
            _lib().orc_free(buf)
        return parse_lean(words) if lean else parse(words)


def parse_lean(words: np.ndarray) -> dict:
    """As parse, with each result's node list as an int32 array and its arc
    list as an int32 array of (src, dst, label) rows."""
    head = [int(x) for x in words[:17]]
    out = {"status": head[0], "n_cg": head[2],
           "stats": [_stats_dict(head[3:10]), _stats_dict(head[10:17])], "results": []}
    p = 17
    for _ in range(head[1]):
        central, sc, sm, key, wsum, nn = (int(x) for x in words[p:p + 6])
        p += 6
        nodes = words[p:p + nn].astype(np.int32)
        p += nn
        na = int(words[p])
        p += 1
        arcs = words[p:p + 3 * na].astype(np.int32).reshape(-1, 3)
        p += 3 * na
        out["results"].append({"central": central, "score_c": sc, "score_m": sm, "key": key,
                               "weight_sum": wsum, "nodes": nodes, "arcs": arcs})
    return out


def parse(words: np.ndarray) -> dict:
    """Decode the oracle's int64 output words."""
    w = [int(x) for x in words]
    out = {"status": w[0], "n_cg": w[2],
           "stats": [_stats_dict(w[3:10]), _stats_dict(w[10:17])], "results": []}
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
