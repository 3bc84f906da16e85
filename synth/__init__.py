"""Seeded synthetic inputs: bi-directed labelled power-law graphs, node weights,
a keyword inverted index and radial-pattern queries.

Stand-ins for the paper's Wikidata dumps and AAAI keyword queries (Section 5.1,
Tables 1-2), which are not available here.  The module holds no part of the
search method's arithmetic; the reference implementation (``oracle``) and the
GPU library both take its arrays unchanged.

Workloads (names follow the sizes they describe):

* ``small``  : 10k nodes, 50k directed edges, power-law 2.1, 100 labels,
               2k-keyword vocabulary, Zipf 1.1, 1-3 keywords per node;
               queries 2 central + 2 marginal from the 200 most frequent
               keywords, k = w = 10, level bound 20.
* ``medium`` : 2M nodes, 20M edges, vocabulary 100k; 3 + 3 keywords,
               k = w = 20, level bound 20.
* ``large``  : 20M nodes, 200M edges, power-law 2.0, four planted hubs with
               1.0/1.2/1.5/2.0M extra out-edges, vocabulary 1M; 5 + 5
               keywords, k = w = 50, level bound 12.
* ``batch``  : 20M nodes, 200M edges with the medium generator settings;
               256 queries with 1-4 central and 1-4 marginal keywords.
* ``serve``  : 50M nodes, 500M edges, vocabulary 1M; 2-10 keywords split
               randomly into central/marginal.
* ``tiny*``  : a few hundred nodes, for brute-force checks.
"""
from __future__ import annotations

import ctypes
import dataclasses
import functools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")


def build(force: bool = True) -> str:
    """Compile the generator into ``synth/libsynth.so`` (gcc, no GPU code)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "synth.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("pl_alpha", ctypes.c_double), ("n_labels", ctypes.c_int32),
                ("vocab", ctypes.c_int32), ("zipf_s", ctypes.c_double),
                ("kw_min", ctypes.c_int32), ("kw_max", ctypes.c_int32),
                ("n_hubs", ctypes.c_int32), ("hub_deg", ctypes.c_int64 * 8),
                ("seed", ctypes.c_uint64), ("abar_sources", ctypes.c_int32),
                ("abar_targets", ctypes.c_int32)]


@functools.lru_cache(maxsize=1)
def _lib():
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.synth_generate.restype = ctypes.c_void_p
    lib.synth_generate.argtypes = [ctypes.POINTER(_Params)]
    lib.synth_sizes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
    lib.synth_copy.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 7
    lib.synth_free.argtypes = [ctypes.c_void_p]
    return lib


@dataclasses.dataclass(frozen=True)
class GraphSpec:
    n_nodes: int
    n_edges: int
    pl_alpha: float = 2.1
    n_labels: int = 100
    vocab: int = 2000
    zipf_s: float = 1.1
    kw_min: int = 1
    kw_max: int = 3
    hubs: tuple = ()
    seed: int = 1
    abar_sources: int = 10
    abar_targets: int = 1000


@dataclasses.dataclass(frozen=True)
class QuerySpec:
    n_queries: int
    n_central: tuple       # (lo, hi) inclusive
    n_marginal: tuple      # (lo, hi) inclusive; (None, None) = split a total
    k: int
    w: int
    max_level: int
    seed: int
    n_total: tuple = None  # (lo, hi): total keywords, split randomly (serving)
    top: int = 200


@dataclasses.dataclass
class Graph:
    """Bi-directed CSR graph; rows sorted by (label, destination)."""
    n_nodes: int
    row_ptr: np.ndarray      # int64 [n+1]
    col: np.ndarray          # int32 [A]
    label: np.ndarray        # uint16 [A]
    node_weight: np.ndarray  # uint8 [n]
    kw_ptr: np.ndarray       # int64 [vocab+1]
    kw_nodes: np.ndarray     # int32, each keyword's nodes ascending
    abar_x100: int
    n_edges: int
    hubs: tuple

    @property
    def n_arcs(self) -> int:
        return int(self.col.shape[0])

    @property
    def vocab(self) -> int:
        return int(self.kw_ptr.shape[0] - 1)

    @property
    def abar(self) -> float:
        return self.abar_x100 / 100.0


@dataclasses.dataclass(frozen=True)
class Query:
    central: tuple
    marginal: tuple
    k: int
    w: int
    max_level: int = 20
    gamma_num: int = 1
    gamma_den: int = 2
    alpha: float = 0.0     # 0: the alpha the graph was loaded with
    score_mode: int = 0    # 0: gamma-weighted sum of S^c and S^m, 1: their product
    rerank: int = 0        # 1: equal scores re-ranked by the sum of arc levels


GRAPHS = {
    "tiny": GraphSpec(300, 900, vocab=40, seed=11, abar_sources=20, abar_targets=100),
    "tiny2": GraphSpec(2000, 8000, vocab=200, seed=12, abar_sources=20, abar_targets=200),
    "small": GraphSpec(10_000, 50_000, vocab=2000, seed=1),
    "medium": GraphSpec(2_000_000, 20_000_000, vocab=100_000, seed=2),
    "large": GraphSpec(20_000_000, 200_000_000, pl_alpha=2.0, vocab=1_000_000, seed=3,
                       hubs=(1_000_000, 1_200_000, 1_500_000, 2_000_000)),
    "batch": GraphSpec(20_000_000, 200_000_000, vocab=100_000, seed=4),
    "serve": GraphSpec(50_000_000, 500_000_000, vocab=1_000_000, seed=5),
}

QUERIES = {
    "tiny": QuerySpec(64, (2, 2), (2, 2), 5, 5, 20, seed=111, top=30),
    "tiny2": QuerySpec(64, (2, 2), (2, 2), 10, 10, 20, seed=112, top=100),
    "small": QuerySpec(64, (2, 2), (2, 2), 10, 10, 20, seed=101),
    "medium": QuerySpec(32, (3, 3), (3, 3), 20, 20, 20, seed=102),
    "large": QuerySpec(8, (5, 5), (5, 5), 50, 50, 12, seed=103),
    "batch": QuerySpec(256, (1, 4), (1, 4), 20, 20, 20, seed=104),
    "serve": QuerySpec(4096, None, None, 20, 20, 20, seed=501, n_total=(2, 10)),
}


@functools.lru_cache(maxsize=2)
def make_graph(name_or_spec) -> Graph:
    spec = GRAPHS[name_or_spec] if isinstance(name_or_spec, str) else name_or_spec
    p = _Params()
    p.n_nodes, p.n_edges, p.pl_alpha = spec.n_nodes, spec.n_edges, spec.pl_alpha
    p.n_labels, p.vocab, p.zipf_s = spec.n_labels, spec.vocab, spec.zipf_s
    p.kw_min, p.kw_max, p.n_hubs = spec.kw_min, spec.kw_max, len(spec.hubs)
    for i, d in enumerate(spec.hubs):
        p.hub_deg[i] = d
    p.seed, p.abar_sources, p.abar_targets = spec.seed, spec.abar_sources, spec.abar_targets
    lib = _lib()
    h = lib.synth_generate(ctypes.byref(p))
    if not h:
        raise RuntimeError(f"graph generation failed for {spec}")
    try:
        sz = (ctypes.c_int64 * 6)()
        lib.synth_sizes(h, sz)
        n, A, nkw, vocab, abar_x100, n_edges = list(sz)
        row_ptr = np.empty(n + 1, np.int64)
        col = np.empty(A, np.int32)
        label = np.empty(A, np.uint16)
        nw = np.empty(n, np.uint8)
        kw_ptr = np.empty(vocab + 1, np.int64)
        kw_nodes = np.empty(nkw, np.int32)
        hubs = np.zeros(8, np.int64)
        lib.synth_copy(h, row_ptr.ctypes.data, col.ctypes.data, label.ctypes.data,
                       nw.ctypes.data, kw_ptr.ctypes.data, kw_nodes.ctypes.data,
                       hubs.ctypes.data)
    finally:
        lib.synth_free(h)
    return Graph(n, row_ptr, col, label, nw, kw_ptr, kw_nodes, int(abar_x100), int(n_edges),
                 tuple(int(x) for x in hubs[:len(spec.hubs)]))


def top_keywords(g: Graph, top: int) -> np.ndarray:
    """The ``top`` most frequent keywords (ties broken by smaller id)."""
    freq = np.diff(g.kw_ptr)
    ids = np.arange(freq.shape[0])
    order = np.lexsort((ids, -freq))
    return order[:top]


def make_queries(g: Graph, qs) -> list:
    """Distinct keywords drawn uniformly from the most frequent ones; the first
    ones drawn are central, the rest marginal (Section 5.2 query generation)."""
    qs = QUERIES[qs] if isinstance(qs, str) else qs
    rng = np.random.Generator(np.random.PCG64(qs.seed))
    pool = top_keywords(g, qs.top)
    out = []
    for _ in range(qs.n_queries):
        if qs.n_total is not None:
            n = int(rng.integers(qs.n_total[0], qs.n_total[1] + 1))
            nc = int(rng.integers(1, n))
            nm = n - nc
        else:
            nc = int(rng.integers(qs.n_central[0], qs.n_central[1] + 1))
            nm = int(rng.integers(qs.n_marginal[0], qs.n_marginal[1] + 1))
        pick = rng.choice(pool, size=nc + nm, replace=False)
        out.append(Query(tuple(int(x) for x in pick[:nc]), tuple(int(x) for x in pick[nc:]),
                         qs.k, qs.w, qs.max_level))
    return out
