"""Pins of the reference implementation's work counters and status bits.

The counters (levels, frontier, e_arc, e_alg, gate_pass, h_writes) are
derived here from the Dial-bucket distances and the frontier rule of
Algorithm 1, never from the oracle's own bookkeeping:

* Frontier Enqueue (Section 4.2.2) takes every flagged node; the level-0
  frontier is the keyword nodes.  A node is flagged for level l+1 when some
  keyword reaches it at level l+1 (the expansion of level l writes l+1 and sets
  its flag, Definition 8), or when it was a frontier at level l, was not
  stopped by the joining flag, and has an arc whose level is above l
  (Algorithm 1 keeps such a node in the frontier: the gate fails).
* The joining flag of a node is set by identification at the level where its
  row becomes complete, so a frontier is stopped at level l exactly when every
  keyword of the run reached it at a level <= l (only when the run blocks).
* Algorithm 1 scans the whole row of every frontier that is not stopped, once
  per keyword whose hitting level is <= l: e_arc adds the degree once, e_alg
  once per such keyword, gate_pass the arcs of level <= l.
* Every hitting level that Algorithm 1 writes is a finite, non-zero entry of H
  (written once, Theorem "lockfree"): h_writes is their number.
* The run's end level: the central run stops at the first level where the
  frontier is empty, where at least w central nodes (complete rows) have been
  found, or at the level bound; the marginal run without Theorem 4 stops when
  every selected CG has an RPG (its level is the largest S^m, Eq. 5).
* Status bit 0 / bit 1: the central / marginal run ended at the level bound.
"""
from __future__ import annotations

import numpy as np
import pytest

import graphs
import oracle
import synth
from test_oracle_pins import INF, dial, rpg_expectation, tiny_cases

COUNTERS = ("levels", "frontier", "e_arc", "e_alg", "gate_pass", "h_writes")


def frontiers(g, act, D, block, last_level):
    """Frontier sets Q_0..Q_last_level from the final distances D (entries
    <= level are the hitting levels known at that level)."""
    n = g.n_nodes
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(n), deg)
    amax = np.zeros(n, np.int64)
    np.maximum.at(amax, src, act.astype(np.int64))
    complete = (D < INF).all(axis=1)
    done_at = np.where(complete, np.where(D < INF, D, -1).max(axis=1), 1 << 30)
    Q = [np.nonzero((D == 0).any(axis=1))[0]]
    for l in range(last_level):
        cur = Q[-1]
        reached = np.nonzero((D == l + 1).any(axis=1))[0]
        stopped = block & (done_at[cur] <= l)
        kept = cur[~stopped & (amax[cur] > l)]
        Q.append(np.union1d(reached, kept))
    return Q, done_at


def derive_counters(g, act, D, block, end_level, expands_at_end=False):
    """Counters of a run that processes levels 0..end_level and expands at
    every level below end_level (identification only at end_level)."""
    deg = np.diff(g.row_ptr).astype(np.int64)
    a = act.astype(np.int64)
    Q, done_at = frontiers(g, act, D, block, end_level)
    c = dict(levels=end_level + 1, frontier=0, e_arc=0, e_alg=0, gate_pass=0, h_writes=0)
    for l, q in enumerate(Q):
        c["frontier"] += len(q)
        if l == end_level and not expands_at_end:
            break
        for f in q:
            if block and done_at[f] <= l:
                continue
            kws = int((D[f] <= l).sum())
            assert kws > 0
            c["e_arc"] += int(deg[f])
            c["e_alg"] += int(deg[f]) * kws
            c["gate_pass"] += int((a[g.row_ptr[f]:g.row_ptr[f + 1]] <= l).sum())
    c["h_writes"] = int(((D > 0) & (D < INF)).sum())
    return c, Q


def central_end(g, D, Q, w, max_level):
    """End level and reason of the central run from the distances: exhausted
    frontier, >= w central nodes (complete rows, identified at their row
    maximum, Theorem identifyCG), or the level bound."""
    complete = (D < INF).all(axis=1)
    rowmax = np.where(complete, D.max(axis=1), 1 << 30)
    for l in range(max_level + 1):
        if len(Q[l]) == 0:
            return l, "exhausted"
        if int((rowmax <= l).sum()) >= w:
            return l, "stop"
    return max_level, "level_bound"


def check_run(got, exp):
    for k in COUNTERS:
        assert got[k] == exp[k], (k, got[k], exp[k])


def central_counters(g, act, kws, w, max_level, block=True):
    """Distances up to the level bound, the end level from them, then the
    counters up to that level."""
    lists = [graphs.keyword_nodes(g, t) for t in kws]
    Dfull = dial(g, act, lists, block, max_level)
    Q, _ = frontiers(g, act, Dfull, block, max_level)
    end, reason = central_end(g, Dfull, Q, w, max_level)
    D = np.where(Dfull <= end, Dfull, INF)
    c, _ = derive_counters(g, act, D, block, end)
    return c, reason


# ------------------------------------------------ exploration alone ---

def test_explore_counters_tiny():
    """orc_explore runs to exhaustion or the bound with no identification."""
    for g, act in tiny_cases(60, seed=21):
        o = oracle.Oracle(g)
        for block in (False, True):
            for L in (1, 2, 20):
                kws = [0, 1, 2]
                H, st = o.explore(act, kws, block=block, max_level=L)
                D = dial(g, act, [graphs.keyword_nodes(g, t) for t in kws], block, L)
                Q, _ = frontiers(g, act, D, block, L)
                end = next((l for l in range(L + 1) if len(Q[l]) == 0), L)
                reason = "exhausted" if len(Q[end]) == 0 else "level_bound"
                Dend = np.where(D <= end, D, INF)
                exp, _ = derive_counters(g, act, Dend, block, end)
                check_run(st, exp)
                assert st["end"] == reason


@pytest.mark.parametrize("block", [False, True])
def test_explore_counters_small(block):
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    for q in synth.make_queries(g, "small")[:4]:
        kws = list(q.central) + list(q.marginal)
        H, st = o.explore(act, kws, block=block, max_level=20)
        D = dial(g, act, [graphs.keyword_nodes(g, t) for t in kws], block, 20)
        Q, _ = frontiers(g, act, D, block, 20)
        end = next((l for l in range(21) if len(Q[l]) == 0), 20)
        exp, _ = derive_counters(g, act, np.where(D <= end, D, INF), block, end)
        check_run(st, exp)


# ------------------------------------------------------ both runs ---

@pytest.mark.parametrize("name", ["tiny2", "small"])
def test_query_counters(name):
    """Central run: end level and counters from the distances.  Marginal run
    without Theorem 4: it ends when every selected CG has an RPG (at the
    largest S^m), at exhaustion or at the bound; with Theorem 4 it ends no
    later, and its counters are those of the frontier rule up to its end."""
    g = synth.make_graph(name)
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    for q in synth.make_queries(g, name)[:8]:
        exp1, reason1 = central_counters(g, act, q.central, q.w, q.max_level)
        full = o.query(act, q, flags=oracle.FLAG_NO_THM4)
        early = o.query(act, q)
        for r in (full, early):
            check_run(r["stats"][0], exp1)
            assert r["stats"][0]["end"] == reason1
            assert bool(r["status"] & 1) == (reason1 == "level_bound")
        # marginal run
        M = list(q.marginal)
        block = len(M) >= 2
        cgs = o.query(act, synth.Query(q.central, (), q.w, q.w, q.max_level))
        if not cgs["results"] or not M:
            assert full["stats"][1]["levels"] == 0
            continue
        cg_nodes = {x["central"]: x["nodes"] for x in cgs["results"]}
        order = [(x["score_c"], x["central"]) for x in cgs["results"]]
        every = rpg_expectation(g, act, synth.Query(q.central, q.marginal, len(order) or 1,
                                                    q.w, q.max_level), cg_nodes, order)
        Dm = dial(g, act, [graphs.keyword_nodes(g, t) for t in M], block, q.max_level)
        Qm, _ = frontiers(g, act, Dm, block, q.max_level)
        exhausted = next((l for l in range(q.max_level + 1) if len(Qm[l]) == 0), None)
        if len(every) == len(order) and order:
            all_at = max(x[4] for x in every)
        else:
            all_at = None
        cands = [(l, r) for l, r in ((exhausted, "exhausted"), (all_at, "stop"),
                                     (q.max_level, "level_bound")) if l is not None]
        end2, reason2 = min(cands, key=lambda x: (x[0], ["exhausted", "stop",
                                                          "level_bound"].index(x[1])))
        exp2, _ = derive_counters(g, act, np.where(Dm <= end2, Dm, INF), block, end2)
        check_run(full["stats"][1], exp2)
        assert full["stats"][1]["end"] == reason2
        assert bool(full["status"] & 2) == (reason2 == "level_bound")
        e2 = early["stats"][1]["levels"] - 1
        assert e2 <= end2
        expe, _ = derive_counters(g, act, np.where(Dm <= e2, Dm, INF), block, e2)
        check_run(early["stats"][1], expe)


# ------------------------------------------------------ level bound ---

def path_graph(n_path, kw_ends):
    """A path 0-1-...-(n_path-1), every arc at level 0; keyword t at node
    kw_ends[t]."""
    edges = [(i, i + 1, 0) for i in range(n_path - 1)]
    return graphs.build(n_path, edges, [[v] for v in kw_ends])


def test_status_bit0_central_level_bound():
    """Central keywords at both ends of a 12-node path: the rows of the middle
    nodes complete at level 6; with level bound 3 the central run ends at the
    bound with no CG (bit 0), with bound 20 it stops after the first CG."""
    g = path_graph(12, [0, 11, 5])
    act = np.zeros(g.n_arcs, np.uint8)
    o = oracle.Oracle(g)
    r = o.query(act, synth.Query((0, 1), (), 1, 1, 3))
    assert r["status"] == 1 and r["results"] == []
    assert r["stats"][0]["end"] == "level_bound" and r["stats"][0]["levels"] == 4
    exp, reason = central_counters(g, act, (0, 1), 1, 3)
    assert reason == "level_bound"
    check_run(r["stats"][0], exp)
    # by hand: level-0 arcs never fail the gate, so a node leaves the frontier
    # after its own level: {0, 11}, {1, 10}, {2, 9}, {3, 8}
    assert r["stats"][0]["frontier"] == 8
    assert r["stats"][0]["h_writes"] == 6
    r = o.query(act, synth.Query((0, 1), (), 1, 1, 20))
    assert r["status"] == 0 and r["stats"][0]["end"] == "stop"
    assert [x["central"] for x in r["results"]] == [5]
    # bound 6 with w = 3: nodes 5 and 6 complete at level 6, fewer than w, so
    # the run still ends at the bound (bit 0) and returns both
    r = o.query(act, synth.Query((0, 1), (), 3, 3, 6))
    assert r["status"] == 1 and r["stats"][0]["end"] == "level_bound"
    assert [x["central"] for x in r["results"]] == [5, 6]
    exp, reason = central_counters(g, act, (0, 1), 3, 6)
    assert reason == "level_bound"
    check_run(r["stats"][0], exp)


def test_status_bit1_marginal_level_bound():
    """Central keyword at node 0 (the CG is node 0 itself, V_C = {0}); two
    paths leave node 0, one of 9 arcs to the first marginal keyword, one of
    10 arcs to the second (no node but 0 is reached by both, so the PTC guard
    stops nothing on the way): with bound 4 the marginal run ends at the
    bound without an RPG (bit 1 only); with bound 20 the RPG has S^m = 10."""
    edges = [(i, i + 1, 0) for i in range(9)] + [(0, 10, 0)] + \
            [(i, i + 1, 0) for i in range(10, 19)]
    g = graphs.build(20, edges, [[0], [9], [19]])
    act = np.zeros(g.n_arcs, np.uint8)
    o = oracle.Oracle(g)
    r = o.query(act, synth.Query((0,), (1, 2), 1, 1, 4))
    assert r["status"] == 2 and r["results"] == []
    st = r["stats"][1]
    assert st["end"] == "level_bound" and st["levels"] == 5
    assert st["frontier"] == 10 and st["h_writes"] == 8
    Dm = dial(g, act, [[9], [19]], True, 4)
    exp, _ = derive_counters(g, act, Dm, True, 4)
    check_run(st, exp)
    r = o.query(act, synth.Query((0,), (1, 2), 1, 1, 20))
    assert r["status"] == 0
    assert [(x["central"], x["score_m"]) for x in r["results"]] == [(0, 10)]


def test_gate_retention_counts():
    """A star whose centre (keyword node) has arcs of levels 0, 2 and 4: it
    stays a frontier while an arc above the level remains, so it is scanned at
    levels 0..3 (e_arc = 4 * 3 arcs), and each leaf is reached at
    (its level + 1)."""
    edges = [(0, 1, 0), (0, 2, 1), (0, 3, 2)]
    g = graphs.build(4, edges, [[0]])
    src, dst, lab, _ = graphs.arcs_of(g)
    lv = {0: 0, 1: 2, 2: 4}
    act = np.array([lv[int(x)] for x in lab], np.uint8)
    o = oracle.Oracle(g)
    H, st = o.explore(act, [0], block=False, max_level=20)
    assert H[:, 0].tolist() == [0, 1, 3, 5]
    # the centre at levels 0-4 (its level-4 arc fails the gate through level 3
    # and is crossed at 4), each leaf once (at levels 1, 3 and 5)
    assert st["e_arc"] == 3 * 5 + 3 and st["levels"] == 7 and st["frontier"] == 8
    exp, _ = derive_counters(g, act, H.astype(np.int64), False, st["levels"] - 1)
    check_run(st, exp)
