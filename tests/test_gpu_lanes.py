"""Concurrent lanes: a batch spread over several lanes and the serving loop
(submit / poll / wait) give, per query, exactly the results of the reference
implementation, whatever lane ran the query and in whatever order the
queries finished."""
from __future__ import annotations

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


@pytest.fixture(scope="module")
def small(raks):
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = synth.make_queries(g, "small")
    exp = [o.query(act, q) for q in qs]
    c = raks.Context(0, lanes=4, batch_mode=raks.RAKS_BATCH_LANES)
    c.load_graph(g, alpha=0.5)
    yield c, qs, exp
    c.close()


def test_batch_on_four_lanes_matches_reference(small):
    c, qs, exp = small
    for _ in range(2):
        got = c.query_batch(qs)
        assert len(got) == len(qs)
        for q, a, b in zip(qs, got, exp):
            assert strip(a) == b, q
    assert c.query_batch([]) == []


def test_serving_matches_reference(small, raks):
    c, qs, exp = small
    c.serve_start(lanes=3)
    try:
        with pytest.raises(raks.RaksError) as e:
            c.query(qs[0])
        assert e.value.code == -4
        tickets = [c.submit(q) for q in qs]
        got = {}
        # take some results as they finish, then wait for the rest
        for i, t in enumerate(tickets[:8]):
            r = c.poll(t)
            if r is not None:
                got[i] = r
        for i, t in enumerate(tickets):
            if i not in got:
                got[i] = c.wait(t)
        for i, q in enumerate(qs):
            assert strip(got[i]) == exp[i], q
            assert got[i]["queue_ms"] >= 0.0 and got[i]["host_ms"] >= got[i]["queue_ms"]
        # a taken ticket is gone; an invalid query fails when it is taken
        with pytest.raises(raks.RaksError) as e:
            c.wait(tickets[0])
        assert e.value.code == -1
        bad = c.submit(synth.Query((1, 1), (), 2, 2))
        with pytest.raises(raks.RaksError) as e:
            c.wait(bad)
        assert e.value.code == -1
    finally:
        c.serve_stop()
    with pytest.raises(raks.RaksError) as e:
        c.submit(qs[0])
    assert e.value.code == -4
    assert strip(c.query(qs[1])) == exp[1]


def test_serve_stop_drains_uncollected(small):
    c, qs, exp = small
    c.serve_start(lanes=2, queue_cap=0)
    for q in qs[:10]:
        c.submit(q)
    c.serve_stop()            # runs and frees the ten queries
    assert strip(c.query(qs[2])) == exp[2]


def test_medium_batch_on_lanes(raks):
    g = synth.make_graph("medium")
    o = oracle.Oracle(g, check=False)
    act = o.activation(g.abar, 0.5)
    qs = synth.make_queries(g, "medium")[6:12]
    c = raks.Context(0, lanes=4, batch_mode=raks.RAKS_BATCH_LANES)
    try:
        c.load_graph(g, alpha=0.5)
        got = c.query_batch(qs)
        for q, a in zip(qs, got):
            assert strip(a) == o.query(act, q), q
    finally:
        c.close()
