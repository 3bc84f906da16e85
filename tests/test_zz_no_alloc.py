"""raks_query_noalloc, the entry point for callers that cannot allocate device
memory, against raks_query (whose kernels it shares) and the reference
implementation: the same results, counters and status bits, bit for bit, on
calls in a row whose inputs shrink (the static scratch keeps the previous
call's contents), and clear errors for what it cannot take."""
from __future__ import annotations

import numpy as np
import pytest

import graphs
import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def raks():
    import paper_2001_06770_amd as raks
    return raks


@pytest.fixture(scope="module")
def ctx(raks):
    c = raks.Context(0)
    yield c
    c.close()


def strip(r):
    r = dict(r)
    for k in ("device_ms", "host_ms", "queue_ms"):
        r.pop(k, None)
    return r


def test_two_calls_in_a_row_match_raks_query(ctx):
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    ctx.load_graph(g, alpha=0.5)
    q0 = synth.make_queries(g, "small")[0]
    pool = [int(t) for t in synth.top_keywords(g, 300) if t not in q0.central + q0.marginal]
    big = synth.Query(q0.central + tuple(pool[:6]), tuple(pool[6:22]), 20, 256)
    small = synth.Query(q0.central[:1], q0.marginal[:1], 1, 1)
    got_big = ctx.query_noalloc(big)
    got_small = ctx.query_noalloc(small)   # right after the larger call
    for q, got in ((big, got_big), (small, got_small)):
        exp = strip(ctx.query(q))
        assert strip(got) == exp, q
        assert exp == strip(o.query(act, q)), q
    assert got_big["results"] and got_small["results"]


def test_every_small_query_then_a_smaller_graph(ctx):
    g = synth.make_graph("small")
    ctx.load_graph(g, alpha=0.5)
    for q in synth.make_queries(g, "small")[:24]:
        assert strip(ctx.query_noalloc(q)) == strip(ctx.query(q)), q
    g2 = synth.make_graph("tiny2")
    o2 = oracle.Oracle(g2)
    act2 = o2.activation(g2.abar, 0.5)
    ctx.load_graph(g2, alpha=0.5)
    for q in synth.make_queries(g2, "tiny2"):
        got = strip(ctx.query_noalloc(q))
        assert got == strip(ctx.query(q)), q
        assert got == strip(o2.query(act2, q)), q


def test_output_arrays_too_small(ctx, raks):
    g = synth.make_graph("small")
    ctx.load_graph(g, alpha=0.5)
    q = synth.make_queries(g, "small")[1]
    exp = strip(ctx.query(q))
    n_nodes = sum(len(r["nodes"]) for r in exp["results"])
    n_arcs = sum(len(r["arcs"]) for r in exp["results"])
    assert n_nodes > 1 and n_arcs > 1
    with pytest.raises(raks.RaksError) as e:
        ctx.query_noalloc(q, cap_nodes=n_nodes - 1, cap_arcs=n_arcs)
    assert e.value.code == -2 and "too small" in str(e.value)
    assert e.value.need == (n_nodes, n_arcs)
    assert strip(ctx.query_noalloc(q, cap_nodes=n_nodes, cap_arcs=n_arcs)) == exp


def test_alpha_levels_must_exist(ctx, raks):
    g = synth.make_graph("small")
    ctx.load_graph(g, alpha=0.5)
    q = synth.make_queries(g, "small")[2]
    qa = synth.Query(q.central, q.marginal, q.k, q.w, alpha=0.3)
    with pytest.raises(raks.RaksError) as e:
        ctx.query_noalloc(qa)
    assert e.value.code == -4
    exp = strip(ctx.query(qa))   # builds the levels for alpha 0.3
    assert strip(ctx.query_noalloc(qa)) == exp


def chain(n):
    """Path 0 - 1 - ... - n-1 with one label; keyword 0 at node 0, keyword 1
    at node n-1."""
    deg = np.full(n, 2, np.int64)
    deg[0] = deg[-1] = 1
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), np.int32)
    col[row_ptr[1:-1]] = np.arange(0, n - 1, dtype=np.int32)          # left neighbours of 1..n-1
    col[row_ptr[1:n] - 1] = np.arange(1, n, dtype=np.int32)           # right neighbours of 0..n-2
    return graphs.G(n, row_ptr, col, np.zeros(col.shape[0], np.uint16), np.zeros(n, np.uint8),
                    np.array([0, 1, 2], np.int64), np.array([0, n - 1], np.int32))


def test_graph_beyond_the_scratch_is_rejected(ctx, raks):
    n = 6_000_000   # the node buffers alone need more than the 256 MiB
    g = chain(n)
    assert (np.diff(g.row_ptr) > 0).all() and g.col[0] == 1 and g.col[-1] == n - 2
    ctx.load_graph(g, alpha=0.5)
    q = synth.Query((0,), (1,), 1, 1)
    with pytest.raises(raks.RaksError) as e:
        ctx.query_noalloc(q)
    assert e.value.code == -2 and "256 MiB scratch" in str(e.value)
    # the entry point still works on a graph that fits
    g2 = synth.make_graph("tiny2")
    ctx.load_graph(g2, alpha=0.5)
    q2 = synth.make_queries(g2, "tiny2")[0]
    assert strip(ctx.query_noalloc(q2)) == strip(ctx.query(q2))
