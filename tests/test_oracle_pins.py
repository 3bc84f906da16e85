"""Pins of the reference implementation (``oracle``) against what the paper and
plain mathematics fix, never against the oracle itself:

* Theorem 1 (bounds of the fine weight given its activation level), the
  special values of Eqs. 1-3 and an independent count of the label degrees;
* Definition 7 path scores by brute-force enumeration of simple paths
  (Theorem "distGlevel": Algorithm 1 fills H with these distances);
* a Dial-bucket (max,+1) label-setting formulation with and without the
  joining-flag blocking, written from the expansion behaviour (Definition 8);
* plain multi-source BFS when every activation level is 0 or uniform;
* order independence of Algorithm 1 (Theorem "lockfree");
* Lemma 1 / Algorithm 2 against brute-force enumeration of the paths whose
  every prefix is a shortest path;
* Theorem 4 against a marginal run without early termination;
* a hand-derived worked example.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import graphs
import oracle
import synth

INF = 255


def round_half_up(v):
    return math.floor(v + 0.5)


# ------------------------------------------------------------ activation ---

def independent_label_counts(g):
    """c_e = |out-arcs of src with label l| + |in-arcs of dst with label l|,
    counted with numpy on the bi-directed arc list."""
    src, dst, lab, _ = graphs.arcs_of(g)
    key_out = src * 65536 + lab
    u, inv, cnt = np.unique(key_out, return_inverse=True, return_counts=True)
    deg_src = cnt[inv]
    key_in = dst * 65536 + lab           # in-arcs of dst with label l
    ui, cnt_in = np.unique(key_in, return_counts=True)
    deg_dst = cnt_in[np.searchsorted(ui, key_in)]
    return deg_src + deg_dst


def theorem1_holds(x, a, abar, alpha, eps=1e-9):
    """Theorem 1: bounds on the rescaled weight x given the level a."""
    ra = round_half_up(abar)
    lo_r = alpha * (a - 0.5) / abar
    hi_r = alpha * (a + 0.5) / abar
    lo_p = 1 + (a - 0.5 - 2 * abar) * (1 - alpha) / abar
    hi_p = 1 + (a + 0.5 - 2 * abar) * (1 - alpha) / abar
    lo = np.where(a < ra, lo_r, np.where(a == ra, lo_r, lo_p))
    hi = np.where(a < ra, hi_r, hi_p)
    return (lo - eps <= x) & (x < hi + eps)


@pytest.mark.parametrize("abar,alpha", [(3.1, 0.5), (3.87, 0.2), (3.68, 0.8), (2.0, 0.5)])
def test_activation_theorem1_edge(abar, alpha):
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act, _, x, c = o.activation(abar, alpha, oracle.MODE_EDGE, want_x=True)
    c_ind = independent_label_counts(g)
    np.testing.assert_array_equal(c, c_ind)
    lc = np.log(c_ind.astype(np.float64))
    x_ind = (lc - lc.min()) / (lc.max() - lc.min())
    np.testing.assert_allclose(x, x_ind, rtol=0, atol=1e-12)
    assert theorem1_holds(x_ind, act.astype(np.int64), abar, alpha).all()
    # the reverse arc has the same label counts, hence the same level
    src, dst, lab, _ = graphs.arcs_of(g)
    rev = np.lexsort((src, lab, dst))            # arcs ordered by (dst, label, src)
    fwd = np.lexsort((dst, lab, src))            # by (src, label, dst) = CSR order
    np.testing.assert_array_equal(act[fwd], act[rev])
    # extremes: the least frequent label pair gets level 0, the most frequent Round(2A)
    assert act[c_ind == c_ind.min()].max() == 0
    assert act[c_ind == c_ind.max()].min() == round_half_up(2 * abar)


def test_activation_node_mode():
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    abar, alpha = 3.1, 0.4
    act, act_node, x, _ = o.activation(abar, alpha, oracle.MODE_NODE, want_x=True)
    nw = g.node_weight.astype(np.float64)
    x_ind = (nw - nw.min()) / (nw.max() - nw.min())
    np.testing.assert_array_equal(x, x_ind)
    assert theorem1_holds(x_ind, act_node.astype(np.int64), abar, alpha).all()
    np.testing.assert_array_equal(act, act_node[g.col])


@pytest.mark.parametrize("abar,alpha", [(3.87, 0.5), (3.68, 0.3), (1.2, 0.9), (5.5, 0.5)])
def test_level_special_values(abar, alpha):
    assert oracle.level_of(0.0, abar, alpha) == 0
    assert oracle.level_of(1.0, abar, alpha) == round_half_up(2 * abar)
    assert oracle.level_of(alpha, abar, alpha) == round_half_up(abar)


def test_level_rounding_is_half_up():
    # x = 0.125, A = 2, alpha = 0.5: v = 2 - 2*0.375/0.5 = 0.5 exactly; Theorem 1
    # puts x = alpha*(a-0.5)/A at the closed lower end of level a = 1.
    assert oracle.level_of(0.125, 2.0, 0.5) == 1
    # penalty side: x = 0.625, A = 2, alpha = 0.5: v = 2 + 2*0.125/0.5 = 2.5 -> 3
    assert oracle.level_of(0.625, 2.0, 0.5) == 3


def test_uniform_weights_give_level_zero():
    # every label pair equally frequent (a cycle with one label): all x = 0
    n = 12
    g = graphs.build(n, [(i, (i + 1) % n, 0) for i in range(n)], [[0]])
    act = oracle.Oracle(g).activation(3.0, 0.5)
    assert (act == 0).all()


# ------------------------------------------- path scores, brute force ---

def path_score(levels):
    """Definition 7, recursively: F(single node) = 0; F(p) = max(F(p-), a) + 1."""
    f = 0
    for a in levels:
        f = max(f, a) + 1
    return f


def test_path_score_closed_form():
    rng = np.random.default_rng(5)
    for _ in range(2000):
        h = int(rng.integers(0, 8))
        a = rng.integers(0, 10, h)
        closed = max([h] + [int(a[j]) + h - j for j in range(h)])  # 0-based j
        assert path_score(a) == closed


def adjacency(g, act):
    src, dst, lab, idx = graphs.arcs_of(g)
    adj = [[] for _ in range(g.n_nodes)]
    for s, d, l, e in zip(src, dst, lab, idx):
        adj[int(s)].append((int(d), int(act[e]), int(l)))
    return adj


def brute_distances(adj, sources):
    """D(t, v) = min over simple paths from V_t of Definition 7 scores."""
    n = len(adj)
    D = [INF] * n

    def dfs(u, f, seen):
        if f < D[u]:
            D[u] = f
        for v, a, _ in adj[u]:
            if v not in seen:
                seen.add(v)
                dfs(v, max(f, a) + 1, seen)
                seen.remove(v)

    for s in sources:
        dfs(s, 0, {s})
    return D


def brute_prefix_optimal(adj, sources, target, D):
    """Union of nodes/arcs of simple paths V_t -> target whose every prefix
    score equals the distance of its end node (the paths Algorithm 2 can
    recover, by Lemma 1)."""
    nodes, arcs = set(), set()

    def dfs(u, f, path_nodes, path_arcs):
        if f != D[u]:
            return
        if u == target:
            nodes.update(path_nodes)
            arcs.update(path_arcs)
            return
        for v, a, l in adj[u]:
            if v not in path_nodes:
                dfs(v, max(f, a) + 1, path_nodes | {v}, path_arcs | {(u, v, l)})

    for s in sources:
        dfs(s, 0, frozenset([s]), frozenset())
    return nodes, arcs


def tiny_cases(count, seed, n_lo=5, n_hi=9):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        m = int(rng.integers(n, 2 * n))
        g = graphs.random_graph(rng, n, m, n_labels=3, n_keywords=4)
        src, dst, lab, _ = graphs.arcs_of(g)
        # symmetric random levels per undirected labelled edge
        lv = {}
        act = np.empty(g.n_arcs, np.uint8)
        for e, (s, d, l) in enumerate(zip(src, dst, lab)):
            k = (min(s, d), max(s, d), l)
            if k not in lv:
                lv[k] = int(rng.integers(0, 5))
            act[e] = lv[k]
        out.append((g, act))
    return out


def test_explore_equals_brute_force_distances():
    for g, act in tiny_cases(60, seed=1):
        o = oracle.Oracle(g)
        adj = adjacency(g, act)
        kws = [0, 1, 2, 3]
        for L in (3, 20):
            H, _ = o.explore(act, kws, block=False, max_level=L)
            for i, t in enumerate(kws):
                D = brute_distances(adj, graphs.keyword_nodes(g, t))
                exp = [d if d <= L else INF for d in D]
                assert list(H[:, i]) == exp


# ---------------------------------------------------- Dial formulation ---

def dial(g, act, kw_lists, block, L):
    """Level-by-level (max,+1) label setting.  An arc u->v relaxes for keyword
    i at level m = max(D[u,i], a) (Definition 8), giving D[v,i] = m+1 if v is
    not yet reached; with blocking, u relaxes only while m is below the level
    at which u became reached by every keyword of the run; relaxation stops
    at the level bound L."""
    n, T = g.n_nodes, len(kw_lists)
    src, dst, _, _ = graphs.arcs_of(g)
    a = act.astype(np.int64)
    D = np.full((n, T), INF, np.int64)
    for i, nodes in enumerate(kw_lists):
        D[nodes, i] = 0
    for m in range(L):
        complete = (D < INF).all(axis=1)
        done_at = np.where(complete, D.max(axis=1), 1 << 30)
        ok = done_at[src] > m if block else np.ones(src.shape[0], bool)
        for i in range(T):
            du = D[src, i]
            sel = (du < INF) & (np.maximum(du, a) == m) & ok & (D[dst, i] == INF)
            D[dst[sel], i] = m + 1
    return D


@pytest.mark.parametrize("block", [False, True])
def test_explore_equals_dial_small(block):
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    for q in synth.make_queries(g, "small")[:6]:
        for kws in (list(q.central), list(q.marginal), list(q.central) + list(q.marginal)):
            H, _ = o.explore(act, kws, block=block, max_level=20)
            D = dial(g, act, [graphs.keyword_nodes(g, t) for t in kws], block, 20)
            np.testing.assert_array_equal(H.astype(np.int64), D)


def test_explore_dial_tiny_blocked():
    for g, act in tiny_cases(60, seed=2):
        o = oracle.Oracle(g)
        for L in (2, 20):
            H, _ = o.explore(act, [0, 1, 2], block=True, max_level=L)
            D = dial(g, act, [graphs.keyword_nodes(g, t) for t in (0, 1, 2)], True, L)
            np.testing.assert_array_equal(H.astype(np.int64), D)


# -------------------------------------------------- BFS special cases ---

def bfs_hops(g, sources):
    A = sp.csr_matrix((np.ones(g.n_arcs), g.col, g.row_ptr), shape=(g.n_nodes, g.n_nodes))
    d = csgraph.shortest_path(A, unweighted=True, indices=sources)
    return np.atleast_2d(d).min(axis=0)


@pytest.mark.parametrize("a0", [0, 2])
def test_uniform_levels_are_bfs_hops(a0):
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = np.full(g.n_arcs, a0, np.uint8)
    kws = list(synth.top_keywords(g, 4))
    H, _ = o.explore(act, kws, block=False, max_level=20)
    for i, t in enumerate(kws):
        hops = bfs_hops(g, graphs.keyword_nodes(g, t))
        exp = np.where(hops == 0, 0, hops + a0)
        exp = np.where(np.isfinite(exp) & (exp <= 20), exp, INF)
        np.testing.assert_array_equal(H[:, i].astype(np.float64), exp)


# ------------------------------------------------- order independence ---

def test_order_independence():
    g = synth.make_graph("tiny2")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = synth.make_queries(g, "tiny2")[:10]
    for q in qs:
        base = o.query(act, q)
        for s in (1, 7, 12345):
            assert o.query(act, q, shuffle=s) == base
        kws = list(q.central) + list(q.marginal)
        H0, st0 = o.explore(act, kws, block=True)
        for s in (3, 99):
            H1, st1 = o.explore(act, kws, block=True, shuffle=s)
            np.testing.assert_array_equal(H0, H1)
            assert st0 == st1


# ----------------------------------------- identification and recovery ---

def cg_candidates(D):
    """Central nodes from a distance matrix: rows with every central keyword
    reached; score = max (Theorem identifyCG), ties by (sum, node id)."""
    complete = (D < INF).all(axis=1)
    nodes = np.nonzero(complete)[0]
    return sorted((int(D[v].max()), int(D[v].sum()), int(v)) for v in nodes)


def test_central_graphs_vs_dial_and_brute_force_unblocked():
    for g, act in tiny_cases(50, seed=3):
        o = oracle.Oracle(g)
        n = g.n_nodes
        q = synth.Query((0, 1), (), k=n, w=n, max_level=20)
        res = o.query(act, q, flags=oracle.FLAG_NO_CG_BLOCK)
        D = dial(g, act, [graphs.keyword_nodes(g, 0), graphs.keyword_nodes(g, 1)], False, 20)
        exp = cg_candidates(D)
        got = [(r["score_c"], r["central"]) for r in res["results"]]
        assert got == [(s, v) for s, _, v in exp]
        adj = adjacency(g, act)
        Db = [brute_distances(adj, graphs.keyword_nodes(g, t)) for t in (0, 1)]
        for r in res["results"]:
            nodes, arcs = {r["central"]}, set()
            for t in (0, 1):
                nn, aa = brute_prefix_optimal(adj, graphs.keyword_nodes(g, t), r["central"], Db[t])
                nodes |= nn
                arcs |= aa
            assert set(r["nodes"]) == nodes
            assert set(r["arcs"]) == arcs
            assert r["key"] == r["score_c"] and r["score_m"] == 0


def test_central_graphs_blocked_vs_dial():
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    for q in synth.make_queries(g, "small")[:12]:
        q0 = synth.Query(q.central, (), q.k, q.w, q.max_level)
        res = o.query(act, q0)
        D = dial(g, act, [graphs.keyword_nodes(g, t) for t in q.central], True, q.max_level)
        exp = cg_candidates(D)[:min(q.k, q.w)]
        assert [(r["score_c"], r["central"]) for r in res["results"]] == [(s, v) for s, _, v in exp]
        # invariants of each CG (totality, connectivity, Lemma 1 on every arc)
        for r in res["results"]:
            nodes = set(r["nodes"])
            for t in q.central:
                assert nodes & set(graphs.keyword_nodes(g, t))
            parent = {v: v for v in nodes}

            def find(v):
                while parent[v] != v:
                    parent[v] = parent[parent[v]]
                    v = parent[v]
                return v
            for s, d, l in r["arcs"]:
                assert s in nodes and d in nodes
                parent[find(s)] = find(d)
                e = g.row_ptr[s] + np.searchsorted(
                    g.label[g.row_ptr[s]:g.row_ptr[s + 1]].astype(np.int64) * (1 << 32)
                    + g.col[g.row_ptr[s]:g.row_ptr[s + 1]], l * (1 << 32) + d)
                assert any(D[d, i] == 1 + max(int(act[e]), int(D[s, i])) for i in range(len(q.central)))
            assert len({find(v) for v in nodes}) == 1


def lemma1_chains(g, act, D, i, target):
    """Union of simple paths V_t -> target along which every arc n -> q meets
    Lemma 1 on the column D[:, i] (h_q = 1 + max(a_nq, h_n)); paths are
    enumerated forward from the nodes at distance 0."""
    adj = adjacency(g, act)
    nodes, arcs = {target}, set()

    def dfs(u, path_nodes, path_arcs):
        if u == target:
            nodes.update(path_nodes)
            arcs.update(path_arcs)
            return
        for v, a, l in adj[u]:
            if v not in path_nodes and D[v, i] == 1 + max(a, int(D[u, i])):
                dfs(v, path_nodes | {v}, path_arcs | {(u, v, l)})

    for s in np.nonzero(D[:, i] == 0)[0]:
        dfs(int(s), frozenset([int(s)]), frozenset())
    return nodes, arcs


def test_central_graphs_blocked_brute_force():
    """With blocking, H is no longer the plain distance; Algorithm 2 then
    recovers exactly the Lemma 1 chains of the blocked H (from the Dial
    formulation), checked by path enumeration."""
    for g, act in tiny_cases(80, seed=6):
        o = oracle.Oracle(g)
        q = synth.Query((0, 1, 2), (), k=4, w=4, max_level=20)
        res = o.query(act, q)
        D = dial(g, act, [graphs.keyword_nodes(g, t) for t in (0, 1, 2)], True, 20)
        exp = cg_candidates(D)[:4]
        assert [(r["score_c"], r["central"]) for r in res["results"]] == [(s, v) for s, _, v in exp]
        for r in res["results"]:
            nodes, arcs = set(), set()
            for i in range(3):
                nn, aa = lemma1_chains(g, act, D, i, r["central"])
                nodes |= nn
                arcs |= aa
            assert set(r["nodes"]) == nodes and set(r["arcs"]) == arcs


def test_worked_example_by_hand():
    """Hand-derived: path 0-1-2-3 with level 3 on 1-2 and a detour 1-4-5-2 of
    level-0 edges.  Keyword t0 at node 0, t1 at node 3.
      t0: D = [0, 1, 4, 5, 2, 3]  (node 2: max(1,3)+1 = 4 direct, 4 via 4,5)
      t1: D = [5, 4, 1, 0, 3, 2]
    Rows complete at levels 5, 4, 4, 5, 3, 3, so with w = 2 run 1 stops at
    level 3 with central nodes 4 and 5 (S^c = 3, sums 5 and 5, ties by id).
    Algorithm 2 from 4: t0 recovers 1->4, 0->1; t1 recovers 5->4, 2->5, 3->2.
    From 5: t0 recovers 4->5, 1->4, 0->1; t1 recovers 2->5, 3->2."""
    edges = [(0, 1, 0), (1, 2, 0), (2, 3, 0), (1, 4, 0), (4, 5, 0), (5, 2, 0)]
    g = graphs.build(6, edges, [[0], [3]])
    src, dst, _, _ = graphs.arcs_of(g)
    act = np.array([3 if {int(s), int(d)} == {1, 2} else 0 for s, d in zip(src, dst)], np.uint8)
    o = oracle.Oracle(g)
    H, _ = o.explore(act, [0, 1], block=False)
    assert H[:, 0].tolist() == [0, 1, 4, 5, 2, 3]
    assert H[:, 1].tolist() == [5, 4, 1, 0, 3, 2]
    res = o.query(act, synth.Query((0, 1), (), k=2, w=2, max_level=20))
    assert [(r["central"], r["score_c"]) for r in res["results"]] == [(4, 3), (5, 3)]
    r4, r5 = res["results"]
    assert r4["nodes"] == (0, 1, 2, 3, 4, 5)
    assert set(r4["arcs"]) == {(0, 1, 0), (1, 4, 0), (3, 2, 0), (2, 5, 0), (5, 4, 0)}
    assert set(r5["arcs"]) == {(0, 1, 0), (1, 4, 0), (4, 5, 0), (3, 2, 0), (2, 5, 0)}
    assert res["stats"][0]["levels"] == 4 and res["stats"][0]["end"] == "stop"
    # one keyword from node 0 alone: both the direct and the detour path to 3
    res1 = o.query(act, synth.Query((0,), (), k=6, w=6, max_level=20),
                   flags=oracle.FLAG_NO_CG_BLOCK)
    at3 = [r for r in res1["results"] if r["central"] == 3][0]
    assert set(at3["arcs"]) == {(0, 1, 0), (1, 2, 0), (1, 4, 0), (4, 5, 0), (5, 2, 0), (2, 3, 0)}


# ------------------------------------------------------------- run 2 ---

def rpg_expectation(g, act, q, cg_nodes_by_central, cg_order):
    """RPGs without early termination, from Dial distances of the marginal
    run: S^m = max_j min_{v in V_C} D_j(v) (Definition 3, Eq. 5)."""
    M = list(q.marginal)
    Dm = dial(g, act, [graphs.keyword_nodes(g, t) for t in M], len(M) >= 2, q.max_level)
    Dc = dial(g, act, [graphs.keyword_nodes(g, t) for t in q.central], True, q.max_level)
    out = []
    for rank, (sc, central) in enumerate(cg_order):
        vc = [v for v in cg_nodes_by_central[central] if (Dc[v] == 0).any()]
        dj = Dm[vc].min(axis=0)
        if (dj < INF).all():
            smv = int(dj.max())
            key = q.gamma_num * sc + (q.gamma_den - q.gamma_num) * smv
            out.append((key, sc, rank, central, smv))
    out.sort()
    return out[:q.k]


@pytest.mark.parametrize("name,n_marginal", [("tiny", 2), ("tiny2", 2), ("small", 2),
                                              ("tiny2", 1), ("small", 1), ("small", 3)])
def test_rpg_vs_dial_and_theorem4(name, n_marginal):
    g = synth.make_graph(name)
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    pool = [int(t) for t in synth.top_keywords(g, 60)]
    qs = synth.make_queries(g, name)[:12]
    if n_marginal != 2:
        rng = np.random.default_rng(n_marginal)
        qs = [synth.Query(q.central, tuple(int(t) for t in rng.choice(
              [t for t in pool if t not in q.central], n_marginal, replace=False)), q.k, q.w,
              q.max_level) for q in qs]
    for q in qs:
        cgs = o.query(act, synth.Query(q.central, (), q.w, q.w, q.max_level))
        cg_nodes = {r["central"]: r["nodes"] for r in cgs["results"]}
        order = [(r["score_c"], r["central"]) for r in cgs["results"]]
        full = o.query(act, q, flags=oracle.FLAG_NO_THM4)
        exp = rpg_expectation(g, act, q, cg_nodes, order)
        got = [(r["key"], r["score_c"], r["central"], r["score_m"]) for r in full["results"]]
        assert got == [(k, s, c, m) for k, s, _, c, m in exp]
        early = o.query(act, q)
        assert early["results"] == full["results"]          # Theorem 4 (gamma < 1)
        assert early["stats"][1]["e_arc"] <= full["stats"][1]["e_arc"]
        for r in full["results"]:
            assert set(cg_nodes[r["central"]]) <= set(r["nodes"])


def test_single_marginal_keyword_recovery_brute_force():
    """|M| = 1 (no PTC blocking): the marginal part is SP(m, V_C), the
    prefix-optimal paths from the keyword to the V_C nodes at distance S^m."""
    checked = 0
    for g, act in tiny_cases(80, seed=4):
        o = oracle.Oracle(g)
        q = synth.Query((0, 1), (2,), k=3, w=3, max_level=20)
        cgs = o.query(act, synth.Query((0, 1), (), 3, 3, 20))
        cg = {r["central"]: r for r in cgs["results"]}
        res = o.query(act, q, flags=oracle.FLAG_NO_THM4)
        adj = adjacency(g, act)
        Dm = brute_distances(adj, graphs.keyword_nodes(g, 2))
        Dc = dial(g, act, [graphs.keyword_nodes(g, 0), graphs.keyword_nodes(g, 1)], True, 20)
        n_rpg = sum(1 for r in cgs["results"]
                    if min(Dm[v] for v in r["nodes"] if (Dc[v] == 0).any()) < INF)
        assert len(res["results"]) == min(n_rpg, q.k)
        for r in res["results"]:
            base = cg[r["central"]]
            vc = [v for v in base["nodes"] if (Dc[v] == 0).any()]
            dmin = min(Dm[v] for v in vc)
            assert r["score_m"] == dmin
            nodes, arcs = set(base["nodes"]), set(base["arcs"])
            for v in vc:
                if Dm[v] == dmin:
                    nn, aa = brute_prefix_optimal(adj, graphs.keyword_nodes(g, 2), v, Dm)
                    nodes |= nn
                    arcs |= aa
            assert set(r["nodes"]) == nodes and set(r["arcs"]) == arcs
            checked += 1
    assert checked > 20


@pytest.mark.parametrize("central,marginal", [((0, 1), (2, 3)), ((0,), (1, 2, 3))])
def test_multi_marginal_recovery_blocked_brute_force(central, marginal):
    """|M| >= 2 (PTC blocking on the marginal run): each RPG is its CG plus,
    per marginal keyword j, the Lemma 1 chains of the blocked marginal H
    (Dial formulation) into the V_C nodes at the minimum D_j (Algorithm 2 on
    the marginal run, Definition 5), checked by path enumeration; S^m and the
    key follow Eq. 5 and Eq. 6."""
    checked = 0
    for g, act in tiny_cases(80, seed=7):
        o = oracle.Oracle(g)
        q = synth.Query(central, marginal, k=4, w=4, max_level=20)
        cgs = o.query(act, synth.Query(central, (), q.w, q.w, q.max_level))
        cg = {r["central"]: r for r in cgs["results"]}
        order = [(r["score_c"], r["central"]) for r in cgs["results"]]
        res = o.query(act, q, flags=oracle.FLAG_NO_THM4)
        exp = rpg_expectation(g, act, q, {c: r["nodes"] for c, r in cg.items()}, order)
        assert [(r["key"], r["central"], r["score_m"]) for r in res["results"]] == \
            [(k, c, m) for k, _, _, c, m in exp]
        Dm = dial(g, act, [graphs.keyword_nodes(g, t) for t in marginal], True, q.max_level)
        Dc = dial(g, act, [graphs.keyword_nodes(g, t) for t in central], True, q.max_level)
        for r in res["results"]:
            base = cg[r["central"]]
            vc = [v for v in base["nodes"] if (Dc[v] == 0).any()]
            nodes, arcs = set(base["nodes"]), set(base["arcs"])
            for j in range(len(marginal)):
                dj = min(int(Dm[v, j]) for v in vc)
                assert dj <= r["score_m"]
                for v in vc:
                    if Dm[v, j] == dj:
                        nn, aa = lemma1_chains(g, act, Dm, j, v)
                        nodes |= nn
                        arcs |= aa
            assert set(r["nodes"]) == nodes and set(r["arcs"]) == arcs
            checked += 1
    assert checked > 20


def test_no_marginal_keywords_returns_central_graphs():
    g = synth.make_graph("tiny2")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    q = synth.make_queries(g, "tiny2")[0]
    r = o.query(act, synth.Query(q.central, (), 4, 10, 20))
    assert len(r["results"]) == 4
    assert all(x["key"] == x["score_c"] for x in r["results"])


def test_empty_keyword_gives_no_results():
    g = synth.make_graph("tiny2")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    freq = np.diff(g.kw_ptr)
    empty = int(np.nonzero(freq == 0)[0][0])
    full = int(np.argmax(freq))
    r = o.query(act, synth.Query((full, empty), (), 5, 5, 20))
    assert r["results"] == [] and r["stats"][0]["end"] == "empty_keyword"


def test_graph_contract_rejections():
    g = graphs.build(4, [(0, 1, 0), (1, 2, 1)], [[0]])
    oracle.Oracle(g)
    for corrupt in ("asym", "self", "order"):
        bad = graphs.build(4, [(0, 1, 0), (0, 2, 0), (1, 2, 1)], [[0]])
        bad.col = bad.col.copy()
        if corrupt == "asym":
            bad.col[0] = 3                    # 0 -> 3 has no reverse arc
        elif corrupt == "self":
            bad.col[0] = 0                    # self-loop
        else:
            bad.col[0], bad.col[1] = bad.col[1], bad.col[0]   # row 0 out of order
        with pytest.raises(ValueError):
            oracle.Oracle(bad)


# ----------------------------------------------------- scoring variants ---
# The multiplicative combination (Section 3.3, "also applicable"), the tie
# re-ranking by the sum of edge weights (Section 3.3), and the linear
# coarsening of Section 3.1.

def arc_levels_sum(g, act, arcs):
    """Sum of the activation levels of the given (src, dst, label) arcs,
    located in the CSR arrays independently of the reference's own code."""
    total = 0
    for s, d, lab in arcs:
        lo, hi = int(g.row_ptr[s]), int(g.row_ptr[s + 1])
        hit = [e for e in range(lo, hi) if int(g.col[e]) == d and int(g.label[e]) == lab]
        assert len(hit) == 1
        total += int(act[hit[0]])
    return total


def with_score(q, score_mode=0, rerank=0, k=None, w=None):
    return synth.Query(q.central, q.marginal, q.k if k is None else k, q.w if w is None else w,
                       q.max_level, q.gamma_num, q.gamma_den, 0.0, score_mode, rerank)


@pytest.mark.parametrize("name,n_marginal", [("tiny2", 2), ("small", 2), ("small", 1),
                                              ("small", 3)])
def test_multiplicative_score_vs_dial_and_theorem4(name, n_marginal):
    """S^r = S^c * S^m from Dial distances; early termination with the
    multiplicative bound gives the same top k as running to the end."""
    g = synth.make_graph(name)
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    pool = [int(t) for t in synth.top_keywords(g, 60)]
    rng = np.random.default_rng(30 + n_marginal)
    qs = synth.make_queries(g, name)[:10]
    qs = [synth.Query(q.central, tuple(int(t) for t in rng.choice(
          [t for t in pool if t not in q.central], n_marginal, replace=False)), q.k, q.w,
          q.max_level) for q in qs]
    for q in qs:
        cgs = o.query(act, synth.Query(q.central, (), q.w, q.w, q.max_level))
        cg_nodes = {r["central"]: r["nodes"] for r in cgs["results"]}
        order = [(r["score_c"], r["central"]) for r in cgs["results"]]
        exp = rpg_expectation(g, act, q, cg_nodes, order)
        exp = sorted((sc * smv, sc, rank, central, smv) for _, sc, rank, central, smv in exp)[:q.k]
        qm = with_score(q, score_mode=1)
        full = o.query(act, qm, flags=oracle.FLAG_NO_THM4)
        got = [(r["key"], r["score_c"], r["central"], r["score_m"]) for r in full["results"]]
        assert got == [(k, s, c, m) for k, s, _, c, m in exp]
        early = o.query(act, qm)
        assert early["results"] == full["results"]
        assert early["stats"][1]["e_arc"] <= full["stats"][1]["e_arc"]


def test_multiplicative_without_marginal_ranks_like_eq6():
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    for q in synth.make_queries(g, "small")[:8]:
        q0 = synth.Query(q.central, (), q.k, q.w, q.max_level)
        a = o.query(act, q0)
        m = o.query(act, with_score(q0, score_mode=1))
        assert [r["central"] for r in a["results"]] == [r["central"] for r in m["results"]]
        assert all(r["key"] == r["score_c"] for r in m["results"])


@pytest.mark.parametrize("score_mode", [0, 1])
@pytest.mark.parametrize("name", ["tiny2", "small"])
def test_rerank_vs_brute_force(name, score_mode):
    """Re-ranking ties: every RPG (run to the end, k = w) ordered by
    (S^r, sum of arc levels, S^c, CG rank), first k; the arc-level sums are
    recomputed from the returned arcs."""
    g = synth.make_graph(name)
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = synth.make_queries(g, name)[:12]
    ties = 0
    for q in qs:
        cgs = o.query(act, synth.Query(q.central, (), q.w, q.w, q.max_level))
        rank_of = {r["central"]: i for i, r in enumerate(cgs["results"])}
        allr = o.query(act, with_score(q, score_mode, k=q.w), flags=oracle.FLAG_NO_THM4)
        rows = []
        for r in allr["results"]:
            ws = arc_levels_sum(g, act, r["arcs"])
            assert ws == r["weight_sum"]
            rows.append((r["key"], ws, r["score_c"], rank_of[r["central"]], r["central"],
                         r["nodes"], r["arcs"]))
        keys = [x[0] for x in rows]
        ties += len(keys) - len(set(keys))
        rows.sort()
        exp = [(k, ws, c, n, a) for k, ws, _, _, c, n, a in rows[:q.k]]
        for flags in (0, oracle.FLAG_NO_THM4):
            got = o.query(act, with_score(q, score_mode, rerank=1), flags=flags)
            assert [(r["key"], r["weight_sum"], r["central"], r["nodes"], r["arcs"])
                    for r in got["results"]] == exp
    assert ties > 0   # the workload has equal scores to re-rank


def test_linear_coarsening_is_alpha_half():
    """A linear map of the rescaled weight onto [0, 2*a_bar] with round half
    up (the 'simple linear mapping' of Section 3.1) equals Eqs. 1-3 at
    alpha = 0.5; computed here from independently counted weights."""
    for name in ("tiny2", "small"):
        g = synth.make_graph(name)
        c = independent_label_counts(g).astype(np.float64)
        x = (np.log(c) - np.log(c.min())) / (np.log(c.max()) - np.log(c.min()))
        lin = np.floor(2.0 * g.abar * x + 0.5).astype(np.int64)
        act = oracle.Oracle(g).activation(g.abar, 0.5)
        close = np.abs(2.0 * g.abar * x - np.round(2.0 * g.abar * x) - 0.5) < 1e-9
        assert np.array_equal(act[~close], lin[~close])
