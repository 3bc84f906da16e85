"""Radial pattern keyword search (RAKS) on MI355X / gfx950.

Thin ctypes binding of ``libraks.so`` (C ABI in ``include/raks.h``): it only
marshals arguments; every step of a query runs in the library's HIP kernels.
PyTorch provides device memory (its caching allocator) and the HIP stream.
There is no CPU fallback: without the built library every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libraks.so")

RAKS_ACT_EDGE, RAKS_ACT_NODE = 0, 1
RAKS_BATCH_COHORT, RAKS_BATCH_LANES = 0, 1
END_NAMES = {0: "none", 1: "exhausted", 2: "stop", 3: "level_bound", 4: "empty_keyword"}
TIMER_EXPAND, TIMER_SCAN, TIMER_CONTROL, TIMER_RECOVER, TIMER_OTHER = range(5)

_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class CtxOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("alloc", _ALLOC),
                ("free", _FREE), ("alloc_user", ctypes.c_void_p), ("mem_budget", ctypes.c_uint64),
                ("lanes", ctypes.c_int32), ("rec_nodes", ctypes.c_uint32),
                ("rec_arcs", ctypes.c_uint32), ("rec_chunks", ctypes.c_uint32),
                ("big_list", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    _fields_ = [("expand_wg_per_cu", ctypes.c_int32), ("admit_below", ctypes.c_int32),
                ("expand_tile", ctypes.c_int32), ("cohort_cols", ctypes.c_int32)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("queue_cap", ctypes.c_int32)]


class GraphDesc(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_arcs", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("label", ctypes.c_void_p), ("node_weight", ctypes.c_void_p),
                ("n_keywords", ctypes.c_int32), ("kw_ptr", ctypes.c_void_p),
                ("kw_nodes", ctypes.c_void_p), ("a_bar", ctypes.c_double),
                ("alpha", ctypes.c_double), ("act_mode", ctypes.c_int32)]


class QueryDesc(ctypes.Structure):
    _fields_ = [("central", ctypes.c_void_p), ("n_central", ctypes.c_int32),
                ("marginal", ctypes.c_void_p), ("n_marginal", ctypes.c_int32),
                ("k", ctypes.c_int32), ("w", ctypes.c_int32), ("gamma_num", ctypes.c_int32),
                ("gamma_den", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("score_mode", ctypes.c_int32),
                ("rerank", ctypes.c_int32)]


class Arc(ctypes.Structure):
    _fields_ = [("src", ctypes.c_int32), ("dst", ctypes.c_int32), ("label", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("central_node", ctypes.c_int32), ("score_c", ctypes.c_int32),
                ("score_m", ctypes.c_int32), ("key", ctypes.c_int64),
                ("weight_sum", ctypes.c_int64), ("n_nodes", ctypes.c_int32), ("nodes", ctypes.POINTER(ctypes.c_int32)),
                ("n_arcs", ctypes.c_int32), ("arcs", ctypes.POINTER(Arc))]


class QueryStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32 * 2), ("end_reason", ctypes.c_int32 * 2),
                ("frontier", ctypes.c_int64 * 2), ("e_arc", ctypes.c_int64 * 2),
                ("e_alg", ctypes.c_int64 * 2), ("gate_pass", ctypes.c_int64 * 2),
                ("h_writes", ctypes.c_int64 * 2), ("n_cg", ctypes.c_int32),
                ("device_ms", ctypes.c_double), ("host_ms", ctypes.c_double),
                ("queue_ms", ctypes.c_double)]


class Results(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("r", ctypes.POINTER(Result)), ("stats", QueryStats),
                ("status", ctypes.c_int32)]


class ResultsBuf(ctypes.Structure):
    _fields_ = [("r", ctypes.POINTER(Result)), ("cap_results", ctypes.c_int32),
                ("nodes", ctypes.POINTER(ctypes.c_int32)), ("cap_nodes", ctypes.c_int64),
                ("arcs", ctypes.POINTER(Arc)), ("cap_arcs", ctypes.c_int64),
                ("n", ctypes.c_int32), ("status", ctypes.c_int32),
                ("n_nodes", ctypes.c_int64), ("n_arcs", ctypes.c_int64), ("stats", QueryStats)]


class KernelTiming(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class RaksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"raks error {code}: {msg}")
        self.code = code


_lib_handle = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        L.raks_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(CtxOpts)]
        L.raks_destroy.argtypes = [ctypes.c_void_p]
        L.raks_load_graph.argtypes = [ctypes.c_void_p, ctypes.POINTER(GraphDesc)]
        L.raks_set_alpha.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.raks_get_activations.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.raks_query.argtypes = [ctypes.c_void_p, ctypes.POINTER(QueryDesc),
                                 ctypes.POINTER(ctypes.POINTER(Results))]
        L.raks_query_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(QueryDesc),
                                         ctypes.POINTER(ResultsBuf)]
        L.raks_query_batch.argtypes = [ctypes.c_void_p, ctypes.POINTER(QueryDesc), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.POINTER(Results))]
        L.raks_results_free.argtypes = [ctypes.POINTER(Results)]
        L.raks_serve_start.argtypes = [ctypes.c_void_p, ctypes.POINTER(ServeOpts)]
        L.raks_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(QueryDesc),
                                  ctypes.POINTER(ctypes.c_uint64)]
        L.raks_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64,
                                ctypes.POINTER(ctypes.POINTER(Results))]
        L.raks_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64,
                                ctypes.POINTER(ctypes.POINTER(Results))]
        L.raks_serve_stop.argtypes = [ctypes.c_void_p]
        L.raks_results_free.restype = None
        L.raks_set_batch_mode.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.raks_set_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(Tuning)]
        L.raks_level_table.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        L.raks_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.raks_get_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(KernelTiming)]
        L.raks_last_error.restype = ctypes.c_char_p
        L.raks_version.restype = ctypes.c_char_p
        _lib_handle = L
    return _lib_handle


EXPORTED = ("raks_create", "raks_destroy", "raks_load_graph", "raks_set_alpha",
            "raks_get_activations", "raks_query", "raks_query_batch", "raks_results_free",
            "raks_serve_start", "raks_submit", "raks_poll", "raks_wait", "raks_serve_stop",
            "raks_set_timing", "raks_get_timing", "raks_last_error", "raks_version",
            "raks_set_batch_mode", "raks_level_table", "raks_set_tuning", "raks_query_noalloc")
RAKS_EAGAIN = -5


def _check(rc):
    if rc != 0:
        raise RaksError(rc, lib().raks_last_error().decode())


class _Owned:
    """Library-owned results (``raks_results*``), freed with
    ``raks_results_free`` when the last array viewing them is gone."""

    def __init__(self, ptr):
        self._ptr = ptr

    def __del__(self):
        try:
            lib().raks_results_free(self._ptr)
        except Exception:  # interpreter shutdown
            pass


class _View:
    """A read-only numpy view of library memory that keeps its owner alive."""

    def __init__(self, owner, addr: int, shape, typestr: str = "<i4"):
        self._owner = owner
        self.__array_interface__ = {"data": (addr, True), "shape": shape,
                                    "typestr": typestr, "version": 3}


def _results_to_dict(res: Results, lean: bool = False, owner=None) -> dict:
    """Results as a dict; nodes and arcs as tuples, or as numpy arrays when
    ``lean`` (no per-element Python objects).  With an ``owner`` (lean only)
    the arrays are views of the library's result lists, which stay allocated
    until the arrays are gone; otherwise they are copies."""
    st = res.stats
    stats = []
    for k in range(2):
        d = {"levels": int(st.levels[k]), "end_reason": int(st.end_reason[k]),
             "frontier": int(st.frontier[k]), "e_arc": int(st.e_arc[k]),
             "e_alg": int(st.e_alg[k]), "gate_pass": int(st.gate_pass[k]),
             "h_writes": int(st.h_writes[k])}
        d["end"] = END_NAMES.get(d["end_reason"], "?")
        stats.append(d)
    out = {"status": int(res.status), "n_cg": int(st.n_cg), "stats": stats, "results": [],
           "device_ms": float(st.device_ms), "host_ms": float(st.host_ms),
           "queue_ms": float(st.queue_ms)}
    for i in range(res.n):
        r = res.r[i]
        if owner is not None and lean and r.n_nodes and r.n_arcs:
            nodes = np.asarray(_View(owner, ctypes.cast(r.nodes, ctypes.c_void_p).value,
                                     (r.n_nodes,)))
            arcs = np.asarray(_View(owner, ctypes.cast(r.arcs, ctypes.c_void_p).value,
                                    (r.n_arcs, 3)))
        else:
            nodes = np.empty(r.n_nodes, np.int32)
            if r.n_nodes:
                ctypes.memmove(nodes.ctypes.data, r.nodes, 4 * r.n_nodes)
            arcs = np.empty((r.n_arcs, 3), np.int32)
            if r.n_arcs:
                ctypes.memmove(arcs.ctypes.data, r.arcs, 12 * r.n_arcs)
        if not lean:
            nodes = tuple(nodes.tolist())
            arcs = tuple(map(tuple, arcs.tolist()))
        out["results"].append({"central": int(r.central_node), "score_c": int(r.score_c),
                               "score_m": int(r.score_m), "key": int(r.key),
                               "weight_sum": int(r.weight_sum),
                               "nodes": nodes, "arcs": arcs})
    return out


def _to_dict_owned(ptr, lean: bool) -> dict:
    """Takes ownership of library results: lean dicts view them (freed when
    the views are gone), others copy them (freed at once)."""
    if lean:
        ptr = ctypes.cast(ptr, ctypes.POINTER(Results))   # its own copy of the address
        owner = _Owned(ptr)
        return _results_to_dict(ptr.contents, True, owner)
    try:
        return _results_to_dict(ptr.contents, False)
    finally:
        lib().raks_results_free(ptr)


class Context:
    """One GPU context holding one graph (``raks_ctx``)."""

    def __init__(self, device: int = 0, use_torch: bool = True, mem_budget: int = 0,
                 lanes: int = 1, rec_caps=(0, 0, 0), big_list: int = 0,
                 batch_mode: int = RAKS_BATCH_COHORT, poison=None):
        """``poison`` (a byte, with ``use_torch``): every device buffer the
        library allocates starts filled with it, so that a read of memory the
        library never wrote gives wrong results instead of the zeros a fresh
        allocation often happens to hold (a debugging aid)."""
        self._keep = []
        opts = CtxOpts()
        opts.device = device
        opts.mem_budget = mem_budget
        opts.lanes = lanes
        opts.rec_nodes, opts.rec_arcs, opts.rec_chunks = (int(x) for x in rec_caps)
        opts.big_list = int(big_list)
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible to torch")
            dev = torch.device("cuda", device)
            stream = torch.cuda.current_stream(dev)
            opts.stream = ctypes.c_void_p(stream.cuda_stream)

            live = {}

            def _alloc(size, _user, _torch=torch, _dev=device, _s=stream):
                try:
                    if poison is None:
                        return _torch.cuda.caching_allocator_alloc(size, _dev, _s)
                    buf = _torch.empty(size, dtype=_torch.uint8, device=dev)
                    buf.fill_(int(poison) & 0xFF)
                    _torch.cuda.synchronize(dev)
                    live[buf.data_ptr()] = buf
                    return buf.data_ptr()
                except Exception:
                    return None

            def _free(ptr, _size, _user, _torch=torch):
                if poison is None:
                    _torch.cuda.caching_allocator_delete(ptr)
                else:
                    live.pop(ptr, None)

            opts.alloc = _ALLOC(_alloc)
            opts.free = _FREE(_free)
            self._keep += [opts.alloc, opts.free, stream]
        self._h = ctypes.c_void_p()
        _check(lib().raks_create(ctypes.byref(self._h), ctypes.byref(opts)))
        if batch_mode != RAKS_BATCH_COHORT:
            self.set_batch_mode(batch_mode)

    def set_tuning(self, expand_wg_per_cu: int = 0, admit_below: int = 32, expand_tile: int = 0,
                   cohort_cols: int = 0):
        """Cohort path parameters (see raks_set_tuning)."""
        t = Tuning(int(expand_wg_per_cu), int(admit_below), int(expand_tile), int(cohort_cols))
        _check(lib().raks_set_tuning(self._h, ctypes.byref(t)))

    def set_batch_mode(self, mode: int):
        """RAKS_BATCH_COHORT (queries share level loops) or RAKS_BATCH_LANES."""
        _check(lib().raks_set_batch_mode(self._h, int(mode)))

    def close(self):
        if self._h:
            lib().raks_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def load_graph(self, g, alpha: float = 0.5, mode: int = RAKS_ACT_EDGE, abar: float = None):
        """``g``: arrays of a bi-directed CSR graph (``synth.Graph`` or alike)."""
        arrs = [np.ascontiguousarray(g.row_ptr, np.int64), np.ascontiguousarray(g.col, np.int32),
                np.ascontiguousarray(g.label, np.uint16),
                np.ascontiguousarray(g.node_weight, np.uint8),
                np.ascontiguousarray(g.kw_ptr, np.int64), np.ascontiguousarray(g.kw_nodes, np.int32)]
        rp, col, lab, nw, kp, kn = arrs
        d = GraphDesc(int(g.n_nodes), int(col.shape[0]), rp.ctypes.data, col.ctypes.data,
                      lab.ctypes.data, nw.ctypes.data, int(kp.shape[0] - 1), kp.ctypes.data,
                      kn.ctypes.data, float(g.abar if abar is None else abar), float(alpha), int(mode))
        _check(lib().raks_load_graph(self._h, ctypes.byref(d)))
        self.n_arcs = int(col.shape[0])

    def set_alpha(self, alpha: float):
        _check(lib().raks_set_alpha(self._h, float(alpha)))

    def activations(self) -> np.ndarray:
        out = np.empty(self.n_arcs, np.uint8)
        _check(lib().raks_get_activations(self._h, out.ctypes.data, self.n_arcs))
        return out

    @staticmethod
    def _desc(q, keep):
        c = np.ascontiguousarray(q.central, np.int32)
        m = np.ascontiguousarray(q.marginal if len(q.marginal) else [0], np.int32)
        keep += [c, m]
        return QueryDesc(c.ctypes.data, len(q.central), m.ctypes.data, len(q.marginal), q.k, q.w,
                         getattr(q, "gamma_num", 1), getattr(q, "gamma_den", 2),
                         getattr(q, "max_level", 20), float(getattr(q, "alpha", 0.0)),
                         int(getattr(q, "score_mode", 0)), int(getattr(q, "rerank", 0)))

    def query(self, q, lean: bool = False) -> dict:
        keep = []
        d = self._desc(q, keep)
        out = ctypes.POINTER(Results)()
        _check(lib().raks_query(self._h, ctypes.byref(d), ctypes.byref(out)))
        return _to_dict_owned(out, lean)

    def query_noalloc(self, q, cap_nodes: int = 1 << 20, cap_arcs: int = 1 << 20,
                      lean: bool = False) -> dict:
        """raks_query_noalloc: the query with no device allocation in the call;
        the result lists go into host arrays of the given capacities."""
        keep = []
        d = self._desc(q, keep)
        cap_r = max(int(q.k), 1)
        res_arr = (Result * cap_r)()
        nodes = np.empty(max(cap_nodes, 1), np.int32)
        arcs = np.empty((max(cap_arcs, 1), 3), np.int32)
        buf = ResultsBuf()
        buf.r = ctypes.cast(res_arr, ctypes.POINTER(Result))
        buf.cap_results = cap_r
        buf.nodes = nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        buf.cap_nodes = int(cap_nodes)
        buf.arcs = ctypes.cast(arcs.ctypes.data, ctypes.POINTER(Arc))
        buf.cap_arcs = int(cap_arcs)
        rc = lib().raks_query_noalloc(self._h, ctypes.byref(d), ctypes.byref(buf))
        if rc != 0:
            err = RaksError(rc, lib().raks_last_error().decode())
            err.need = (int(buf.n_nodes), int(buf.n_arcs))
            raise err
        view = Results(buf.n, buf.r, buf.stats, buf.status)
        return _results_to_dict(view, lean)

    def query_batch(self, qs, lean: bool = False) -> list:
        """Runs the queries together (cohorts, or lanes in RAKS_BATCH_LANES mode)."""
        keep = []
        n = len(qs)
        arr = (QueryDesc * max(n, 1))(*[self._desc(q, keep) for q in qs])
        outs = (ctypes.POINTER(Results) * max(n, 1))()
        _check(lib().raks_query_batch(self._h, arr, n, outs))
        res = []
        try:
            for i in range(n):
                ptr = ctypes.cast(outs[i], ctypes.POINTER(Results))
                outs[i] = None   # owned by ptr from here on
                res.append(_to_dict_owned(ptr, lean))
        finally:
            for i in range(n):
                if outs[i]:
                    lib().raks_results_free(outs[i])
        return res

    # ---- serving

    def serve_start(self, lanes: int = 0, queue_cap: int = 0):
        o = ServeOpts(lanes, queue_cap)
        _check(lib().raks_serve_start(self._h, ctypes.byref(o)))

    def submit(self, q) -> int:
        keep = []
        d = self._desc(q, keep)
        t = ctypes.c_uint64()
        _check(lib().raks_submit(self._h, ctypes.byref(d), ctypes.byref(t)))
        return int(t.value)

    def _take(self, fn, ticket: int, lean: bool):
        out = ctypes.POINTER(Results)()
        rc = fn(self._h, ctypes.c_uint64(ticket), ctypes.byref(out))
        if rc == RAKS_EAGAIN:
            return None
        _check(rc)
        return _to_dict_owned(out, lean)

    def poll(self, ticket: int, lean: bool = False):
        """Results of a finished query, or None while it runs."""
        return self._take(lib().raks_poll, ticket, lean)

    def wait(self, ticket: int, lean: bool = False) -> dict:
        return self._take(lib().raks_wait, ticket, lean)

    def serve_stop(self):
        _check(lib().raks_serve_stop(self._h))

    def set_timing(self, enable=True):
        """True: time every kernel group; False: off; an int: mask of timer ids."""
        mask = 0x1F if enable is True else (0 if enable is False else int(enable))
        _check(lib().raks_set_timing(self._h, mask))

    def timing(self, kernel: int) -> dict:
        t = KernelTiming()
        _check(lib().raks_get_timing(self._h, kernel, ctypes.byref(t)))
        return {"launches": int(t.launches), "ms": float(t.ms), "bytes": float(t.bytes)}


def level_table(mode: int, lo: int, hi: int, abar: float, alpha: float) -> np.ndarray:
    """Host-built activation levels of the values lo..hi (label counts in EDGE
    mode, node weights in NODE mode), as the library uses them."""
    out = np.empty(hi - lo + 1, np.uint8)
    _check(lib().raks_level_table(int(mode), int(lo), int(hi), float(abar), float(alpha),
                                  out.ctypes.data))
    return out


def version() -> str:
    return lib().raks_version().decode()
