"""Per-query alpha (the granularity of Eqs. 1-2 chosen per search without
reloading the graph): a query with its own alpha gives exactly the reference
implementation's results on activation levels computed for that alpha, in
EDGE and NODE mode, through the view cache (more alphas than it holds) and
in a batch that mixes alphas over four lanes."""
from __future__ import annotations

import dataclasses

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
def small():
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    return g, o, synth.make_queries(g, "small")


def with_alpha(q, a):
    return dataclasses.replace(q, alpha=a)


@pytest.mark.parametrize("mode", [0, 1], ids=["edge", "node"])
def test_query_alpha_matches_reference(raks, small, mode):
    g, o, qs = small
    c = raks.Context(0)
    try:
        c.load_graph(g, alpha=0.5, mode=mode)
        for a in (0.2, 0.8, 0.35):
            act = o.activation(g.abar, a, mode)
            if mode == oracle.MODE_NODE:
                act = act[0]
            for q in qs[:12]:
                assert strip(c.query(with_alpha(q, a))) == o.query(act, q), (a, q)
        # the context's own alpha, given explicitly or not
        act = o.activation(g.abar, 0.5, mode)
        if mode == oracle.MODE_NODE:
            act = act[0]
        for q in qs[:4]:
            assert strip(c.query(with_alpha(q, 0.5))) == strip(c.query(q)) == o.query(act, q)
    finally:
        c.close()


def test_view_cache_and_mixed_batch(raks, small):
    g, o, qs = small
    alphas = [0.1, 0.25, 0.4, 0.6, 0.75, 0.9]   # more than the cache holds
    acts = {a: o.activation(g.abar, a) for a in alphas}
    c = raks.Context(0, lanes=4)
    try:
        c.load_graph(g, alpha=0.5)
        for _ in range(2):
            for a in alphas:
                q = qs[int(a * 40)]
                assert strip(c.query(with_alpha(q, a))) == o.query(acts[a], q), (a, q)
        mixed = [with_alpha(q, alphas[i % len(alphas)]) for i, q in enumerate(qs[:36])]
        got = c.query_batch(mixed)
        for i, (q, r) in enumerate(zip(qs[:36], got)):
            assert strip(r) == o.query(acts[alphas[i % len(alphas)]], q), (i, q)
        for bad in (1.0, -0.1, 1.5):
            with pytest.raises(raks.RaksError) as e:
                c.query(with_alpha(qs[0], bad))
            assert e.value.code == -1
    finally:
        c.close()
