"""GPU parity: the gfx950 library (through its C ABI) against the reference
implementation, on the same seeded inputs.  Everything is integer once the
activation levels are set, so the bar is bit-exact equality of the activation
levels, of every result (central node, S^c, S^m, key, nodes, arcs), of the
status bits and of the per-run work counters."""
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
    """Drops the timing fields, which differ between runs."""
    r = dict(r)
    for k in ("device_ms", "host_ms", "queue_ms"):
        r.pop(k, None)
    return r


def assert_same(got, exp, q):
    got = strip(got)
    assert got["status"] == exp["status"], q
    assert got["n_cg"] == exp["n_cg"], q
    assert got["stats"] == exp["stats"], (q, got["stats"], exp["stats"])
    assert len(got["results"]) == len(exp["results"]), q
    for i, (a, b) in enumerate(zip(got["results"], exp["results"])):
        assert a == b, (q, i, {k: (a[k], b[k]) for k in a if a[k] != b[k] and k not in ("nodes", "arcs")})
    assert got == exp


def reference(g, mode=oracle.MODE_EDGE, alpha=0.5, check=True):
    o = oracle.Oracle(g, check=check)
    act = o.activation(g.abar, alpha, mode)
    if mode == oracle.MODE_NODE:
        act = act[0]
    return o, act


@pytest.mark.parametrize("mode", [0, 1], ids=["edge", "node"])
@pytest.mark.parametrize("name", ["tiny", "tiny2", "small"])
def test_query_parity(ctx, name, mode):
    g = synth.make_graph(name)
    o, act = reference(g, mode)
    ctx.load_graph(g, alpha=0.5, mode=mode)
    np.testing.assert_array_equal(ctx.activations(), act)
    for q in synth.make_queries(g, name):
        assert_same(ctx.query(q), o.query(act, q), q)


@pytest.mark.parametrize("alpha", [0.2, 0.8])
def test_set_alpha_parity(ctx, alpha):
    g = synth.make_graph("small")
    o, act = reference(g, alpha=alpha)
    ctx.load_graph(g, alpha=0.5)
    ctx.set_alpha(alpha)
    np.testing.assert_array_equal(ctx.activations(), act)
    for q in synth.make_queries(g, "small")[:16]:
        assert_same(ctx.query(q), o.query(act, q), q)


def _variants(g, base):
    pool = [int(t) for t in synth.top_keywords(g, 300)]
    rng = np.random.default_rng(7)
    out = []
    for q in base:
        rest = [t for t in pool if t not in q.central + q.marginal]
        out += [
            synth.Query(q.central, (), q.k, q.w),                                # no marginal keywords
            synth.Query(q.central, q.marginal[:1], q.k, q.w),                    # |M| = 1
            synth.Query(q.central, q.marginal, 1, 1),                            # k = w = 1
            synth.Query(q.central, q.marginal, 3, 17),                           # w > k
            synth.Query(q.central, q.marginal, q.k, q.w, max_level=1),           # level bound
            synth.Query(q.central, q.marginal, q.k, q.w, max_level=2),
            synth.Query(q.central, q.marginal, q.k, q.w, gamma_num=0, gamma_den=1),
            synth.Query(q.central, q.marginal, q.k, q.w, gamma_num=1, gamma_den=1),
            synth.Query(q.central, q.marginal, q.k, q.w, gamma_num=3, gamma_den=4),
            synth.Query(q.central[:1], tuple(rng.choice(rest, 5, replace=False).tolist()), 6, 40),
            synth.Query(tuple(rng.choice(rest, 9, replace=False).tolist()), q.marginal, 4, 8),
            synth.Query(tuple(rng.choice(rest, 16, replace=False).tolist()), (), 5, 5),
            synth.Query(q.central, tuple(rng.choice(rest, 16, replace=False).tolist()), 20, 256),
        ]
    return out


@pytest.mark.parametrize("name", ["tiny2", "small"])
def test_parameter_edge_cases(ctx, name):
    g = synth.make_graph(name)
    o, act = reference(g)
    ctx.load_graph(g, alpha=0.5)
    for q in _variants(g, synth.make_queries(g, name)[:6]):
        assert_same(ctx.query(q), o.query(act, q), q)


def test_empty_keyword_and_isolated_nodes(ctx):
    g = synth.make_graph("tiny2")
    o, act = reference(g)
    ctx.load_graph(g, alpha=0.5)
    freq = np.diff(g.kw_ptr)
    empty = int(np.nonzero(freq == 0)[0][0])
    full = [int(t) for t in synth.top_keywords(g, 4)]
    for q in (synth.Query((full[0], empty), (full[1],), 5, 5),
              synth.Query((full[0],), (empty, full[1]), 5, 5),
              synth.Query((full[0], full[1]), (full[2], empty), 5, 5)):
        got = ctx.query(q)
        assert got["results"] == []
        assert_same(got, o.query(act, q), q)
    # keywords on isolated nodes only
    deg = np.diff(g.row_ptr)
    iso = set(np.nonzero(deg == 0)[0].tolist())
    only_iso = [t for t in range(g.vocab) if freq[t] > 0 and
                set(g.kw_nodes[g.kw_ptr[t]:g.kw_ptr[t + 1]].tolist()) <= iso]
    if only_iso:
        q = synth.Query((only_iso[0], full[0]), (full[1],), 5, 5)
        assert_same(ctx.query(q), o.query(act, q), q)


def test_hand_built_graphs(ctx):
    rng = np.random.default_rng(3)
    for i in range(30):
        n = int(rng.integers(6, 40))
        g = graphs.random_graph(rng, n, int(rng.integers(n, 3 * n)), n_labels=4, n_keywords=6,
                                kw_size=(1, 4))
        g.abar_x100 = int(rng.integers(150, 500))
        mode = i % 2
        o, act = reference(g, mode=mode, alpha=float(rng.uniform(0.2, 0.8)))
        ctx.load_graph(g, alpha=float(rng.uniform(0.2, 0.8)), mode=mode)
        ctx.set_alpha(0.5)
        o, act = reference(g, mode=mode, alpha=0.5)
        np.testing.assert_array_equal(ctx.activations(), act)
        for q in (synth.Query((0, 1), (2, 3), 3, 5), synth.Query((0, 1, 2), (3,), 2, 4),
                  synth.Query((4,), (0, 1, 2, 3, 5), 4, 4), synth.Query((0, 5), (), 6, 6)):
            assert_same(ctx.query(q), o.query(act, q), q)


def test_invalid_inputs_rejected(ctx, raks):
    g = synth.make_graph("tiny")
    ctx.load_graph(g, alpha=0.5)
    bad = [synth.Query((1, 1), (), 2, 2), synth.Query((1, 2), (2,), 2, 2),
           synth.Query((1,), (), 0, 2), synth.Query((1,), (), 3, 2),
           synth.Query((1,), (), 2, 257), synth.Query(tuple(range(17)), (), 2, 2),
           synth.Query((10**6,), (), 2, 2), synth.Query((), (1,), 2, 2),
           synth.Query((1,), (), 2, 2, max_level=251),
           synth.Query((1,), (), 2, 2, gamma_num=3, gamma_den=2)]
    for q in bad:
        with pytest.raises(raks.RaksError) as e:
            ctx.query(q)
        assert e.value.code == -1
    for corrupt in ("asym", "order", "self"):
        b = graphs.build(5, [(0, 1, 0), (0, 2, 0), (1, 2, 1), (3, 4, 2)], [[0], [1]])
        b.col = b.col.copy()
        if corrupt == "asym":
            b.col[0] = 3
        elif corrupt == "order":
            b.col[0], b.col[1] = b.col[1], b.col[0]
        else:
            b.col[0] = 0
        with pytest.raises(raks.RaksError) as e:
            ctx.load_graph(b, alpha=0.5)
        assert e.value.code == -1
    with pytest.raises(raks.RaksError):
        ctx.load_graph(g, alpha=1.0)


def test_repeatable_and_batch_equals_single(ctx):
    g = synth.make_graph("small")
    ctx.load_graph(g, alpha=0.5)
    qs = synth.make_queries(g, "small")[:12]
    single = [strip(ctx.query(q)) for q in qs]
    for _ in range(2):
        assert [strip(ctx.query(q)) for q in qs] == single
    assert [strip(r) for r in ctx.query_batch(qs)] == single


@pytest.fixture(scope="module")
def medium():
    g = synth.make_graph("medium")
    o, act = reference(g, check=False)
    return g, o, act


@pytest.mark.parametrize("qi", range(32))
def test_medium_parity(ctx, medium, qi):
    g, o, act = medium
    if qi == 0:
        ctx.load_graph(g, alpha=0.5)
        np.testing.assert_array_equal(ctx.activations(), act)
    elif getattr(ctx, "n_arcs", None) != g.n_arcs:
        ctx.load_graph(g, alpha=0.5)
    q = synth.make_queries(g, "medium")[qi]
    assert_same(ctx.query(q), o.query(act, q), q)


def test_timing_mask(ctx, raks):
    g = synth.make_graph("small")
    ctx.load_graph(g, alpha=0.5)
    q = synth.make_queries(g, "small")[0]
    ctx.set_timing(1 << raks.TIMER_EXPAND)
    ctx.query(q)
    t = [ctx.timing(i) for i in range(5)]
    ctx.set_timing(False)
    assert t[raks.TIMER_EXPAND]["launches"] > 0 and t[raks.TIMER_EXPAND]["bytes"] > 0
    assert all(t[i]["launches"] == 0 for i in range(5) if i != raks.TIMER_EXPAND)
    ctx.set_timing(True)
    ctx.query(q)
    assert all(ctx.timing(i)["launches"] > 0 for i in (raks.TIMER_EXPAND, raks.TIMER_SCAN,
                                                       raks.TIMER_CONTROL, raks.TIMER_RECOVER))
    ctx.set_timing(False)
    with pytest.raises(raks.RaksError) as e:
        ctx.set_timing(64)
    assert e.value.code == -1
