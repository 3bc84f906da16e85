"""The cohort path (many queries in one level loop, query-tagged hitting-level
matrix, continuous admission) gives, per query, exactly the reference
implementation's results: status, counters of both runs and every result.
Covered: more queries than slots and columns (admission as queries finish),
uneven keyword counts (|C| 1-4, |M| 0-4), the level bound, gamma, the
multiplicative score and re-ranking, NODE activation, the medium workload's
whole query set, and serving (queries submitted while others run)."""
from __future__ import annotations

import random

import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def strip(r):
    r = dict(r)
    for k in ("device_ms", "host_ms", "queue_ms"):
        r.pop(k, None)
    return r


@pytest.fixture(scope="module")
def raks():
    import paper_2001_06770_amd as raks
    return raks


def mixed_queries(g, n, seed, top=100):
    """Queries with 1-4 central and 0-4 marginal keywords and varied parameters."""
    rnd = random.Random(seed)
    pool = [int(x) for x in synth.top_keywords(g, top)]
    out = []
    for i in range(n):
        nc, nm = rnd.randint(1, 4), rnd.randint(0, 4)
        kws = rnd.sample(pool, nc + nm)
        k = rnd.randint(1, 12)
        w = k + rnd.randint(0, 8)
        out.append(synth.Query(tuple(kws[:nc]), tuple(kws[nc:]), k, w,
                               max_level=rnd.choice([1, 2, 3, 20]),
                               gamma_num=rnd.choice([0, 1, 1, 3]), gamma_den=4,
                               score_mode=1 if i % 7 == 3 else 0,
                               rerank=1 if i % 5 == 2 else 0))
    return out


def check(got, exp, qs):
    assert len(got) == len(exp)
    for q, a, b in zip(qs, got, exp):
        assert strip(a) == b, q


def test_cohort_small_all_queries(raks):
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = synth.make_queries(g, "small")
    exp = [o.query(act, q) for q in qs]
    with raks.Context(0) as c:
        c.load_graph(g, alpha=0.5)
        for rep in range(2):
            print(f"[cohort] small batch, pass {rep}", flush=True)
            check(c.query_batch(qs), exp, qs)
        # cohort results equal the single-query path's
        for q, e in zip(qs[:8], exp[:8]):
            assert strip(c.query(q)) == e
        assert c.query_batch([]) == []


@pytest.mark.parametrize("name", ["tiny2", "small"])
def test_cohort_mixed_shapes(raks, name):
    g = synth.make_graph(name)
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = mixed_queries(g, 96, seed=7)
    exp = [o.query(act, q) for q in qs]
    with raks.Context(0) as c:
        c.load_graph(g, alpha=0.5)
        print(f"[cohort] {name} mixed shapes", flush=True)
        check(c.query_batch(qs), exp, qs)


@pytest.mark.parametrize("cols", [16, 32])
def test_cohort_narrow_widths(raks, cols):
    """A cohort of 16 or 32 columns (2- or 4-byte reached masks, fewer queries
    at once), then back to 64 in the same context: same results."""
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = mixed_queries(g, 48, seed=11)
    exp = [o.query(act, q) for q in qs]
    with raks.Context(0) as c:
        c.load_graph(g, alpha=0.5)
        print(f"[cohort] small, {cols} columns", flush=True)
        c.set_tuning(cohort_cols=cols)
        check(c.query_batch(qs), exp, qs)
        c.set_tuning(cohort_cols=64)
        check(c.query_batch(qs[:16]), exp[:16], qs[:16])
        with pytest.raises(raks.RaksError):
            c.set_tuning(cohort_cols=48)


def test_cohort_node_mode(raks):
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5, oracle.MODE_NODE)[0]
    qs = synth.make_queries(g, "small")[:32]
    exp = [o.query(act, q) for q in qs]
    with raks.Context(0) as c:
        c.load_graph(g, alpha=0.5, mode=raks.RAKS_ACT_NODE)
        print("[cohort] small NODE mode", flush=True)
        check(c.query_batch(qs), exp, qs)


def test_cohort_medium_all_queries(raks):
    g = synth.make_graph("medium")
    o = oracle.Oracle(g, check=False)
    act = o.activation(g.abar, 0.5)
    qs = synth.make_queries(g, "medium")
    print("[cohort] medium: reference ...", flush=True)
    exp = [o.query(act, q) for q in qs]
    with raks.Context(0) as c:
        c.load_graph(g, alpha=0.5)
        print("[cohort] medium batch", flush=True)
        check(c.query_batch(qs), exp, qs)
    synth.make_graph.cache_clear()


def test_cohort_serving(raks):
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = synth.make_queries(g, "small") + mixed_queries(g, 32, seed=11)
    exp = [o.query(act, q) for q in qs]
    with raks.Context(0) as c:
        c.load_graph(g, alpha=0.5)
        c.serve_start()
        try:
            print("[cohort] serving", flush=True)
            tickets = [c.submit(q) for q in qs[:40]]
            got = {}
            for i, t in enumerate(tickets[:8]):
                r = c.poll(t)
                if r is not None:
                    got[i] = r
            # more queries arrive while the first ones run
            tickets += [c.submit(q) for q in qs[40:]]
            for i, t in enumerate(tickets):
                if i not in got:
                    got[i] = c.wait(t)
            for i, q in enumerate(qs):
                assert strip(got[i]) == exp[i], q
                assert got[i]["queue_ms"] >= 0.0 and got[i]["host_ms"] >= got[i]["queue_ms"]
            with pytest.raises(raks.RaksError) as e:
                c.wait(tickets[0])
            assert e.value.code == -1
            bad = c.submit(synth.Query((1, 1), (), 2, 2))
            with pytest.raises(raks.RaksError) as e:
                c.wait(bad)
            assert e.value.code == -1
        finally:
            c.serve_stop()
        assert strip(c.query(qs[1])) == exp[1]
        # serving again after a stop, and a stop with results never taken
        c.serve_start()
        for q in qs[:10]:
            c.submit(q)
        c.serve_stop()
        check(c.query_batch(qs[:6]), exp[:6], qs[:6])
