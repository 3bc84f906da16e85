"""Small hand-made and random graphs for the checks, built directly in the
input contract (bi-directed CSR, rows sorted by (label, destination))."""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class G:
    n_nodes: int
    row_ptr: np.ndarray
    col: np.ndarray
    label: np.ndarray
    node_weight: np.ndarray
    kw_ptr: np.ndarray
    kw_nodes: np.ndarray
    abar_x100: int = 300

    @property
    def n_arcs(self):
        return int(self.col.shape[0])

    @property
    def abar(self):
        return self.abar_x100 / 100.0


def build(n, edges, keywords, node_weight=None, abar_x100=300):
    """``edges``: iterable of (u, v, label), made bi-directed here;
    ``keywords``: list of node lists, one per keyword id."""
    arcs = set()
    for u, v, lab in edges:
        if u == v:
            continue
        arcs.add((u, lab, v))
        arcs.add((v, lab, u))
    arcs = sorted(arcs)
    row_ptr = np.zeros(n + 1, np.int64)
    for u, _, _ in arcs:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.int64)
    col = np.array([a[2] for a in arcs], np.int32)
    label = np.array([a[1] for a in arcs], np.uint16)
    kw_ptr = np.zeros(len(keywords) + 1, np.int64)
    kw_nodes = []
    for t, nodes in enumerate(keywords):
        s = sorted(set(nodes))
        kw_nodes.extend(s)
        kw_ptr[t + 1] = kw_ptr[t] + len(s)
    nw = (np.zeros(n, np.uint8) if node_weight is None else np.asarray(node_weight, np.uint8))
    return G(n, row_ptr, col, label, nw, kw_ptr, np.array(kw_nodes, np.int32), abar_x100)


def random_graph(rng, n, m, n_labels=3, n_keywords=4, kw_size=(1, 3)):
    edges = set()
    while len(edges) < m:
        u, v = rng.integers(0, n, 2)
        if u != v:
            edges.add((int(u), int(v), int(rng.integers(0, n_labels))))
    kws = [list(rng.choice(n, size=int(rng.integers(kw_size[0], kw_size[1] + 1)), replace=False))
           for _ in range(n_keywords)]
    nw = rng.integers(0, 60, n)
    return build(n, sorted(edges), kws, node_weight=nw)


def arcs_of(g):
    """(src, dst, label, index) per arc."""
    src = np.repeat(np.arange(g.n_nodes), np.diff(g.row_ptr))
    return src, g.col.astype(np.int64), g.label.astype(np.int64), np.arange(g.n_arcs)


def keyword_nodes(g, t):
    return [int(x) for x in g.kw_nodes[g.kw_ptr[t]:g.kw_ptr[t + 1]]]
