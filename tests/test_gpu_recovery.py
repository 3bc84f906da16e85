"""Recovery capacity growth and the bitmap path for large results: contexts
that start with tiny recovery capacities (1-64 nodes, arcs and work chunks
per instance), or that send every result with more than a few list entries
through the bitmap merge, must still give the reference implementation's
results exactly.  This exercises the per-instance growth, the switch from a
node table to a node bitmap, the repeat of only the CG phase or only the RPG
phase, the bitmap merge of CGs (with V_C) and of RPGs, and a batch of such
queries over two lanes."""
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


@pytest.mark.parametrize("caps,big", [((1, 1, 1), 0), ((8, 8, 4), 0), ((64, 2, 1), 0),
                                      ((0, 0, 0), 4), ((8, 8, 4), 16)],
                         ids=["1-1-1", "8-8-4", "64-2-1", "bitmap4", "8-8-4-bitmap16"])
@pytest.mark.parametrize("name", ["tiny2", "small"])
def test_tiny_capacities_match_reference(raks, name, caps, big):
    g = synth.make_graph(name)
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = synth.make_queries(g, name)[:24]
    c = raks.Context(0, lanes=2, rec_caps=caps, big_list=big)
    try:
        c.load_graph(g, alpha=0.5)
        exp = [o.query(act, q) for q in qs]
        for q, e in zip(qs, exp):
            assert strip(c.query(q)) == e, (caps, q)
        for q, r, e in zip(qs, c.query_batch(qs), exp):
            assert strip(r) == e, (caps, q)
    finally:
        c.close()


def shape_mix(g, n, seed):
    """Queries of 1-4 central and 0-4 marginal keywords with varied k and w,
    so that consecutive queries on a lane need label arrays of different
    sizes in each phase."""
    import random
    rnd = random.Random(seed)
    pool = [int(x) for x in synth.top_keywords(g, 80)]
    out = []
    for _ in range(n):
        nc, nm = rnd.randint(1, 4), rnd.randint(0, 4)
        kws = rnd.sample(pool, nc + nm)
        k = rnd.randint(1, 16)
        out.append(synth.Query(tuple(kws[:nc]), tuple(kws[nc:]), k, k + rnd.randint(0, 16)))
    return out


@pytest.mark.parametrize("poison", [0xFF, 0x5A], ids=["ff", "5a"])
def test_poisoned_memory_labelled_recovery(raks, poison):
    """Every device buffer of the library starts filled with a non-zero byte,
    and recovery starts from one-entry capacities, so that both phases switch
    to labelled searches whose label arrays grow between the phases and
    between queries of different keyword counts.  Results still equal the
    reference's, one query at a time and as cohort batches: a label word the
    library never cleared would make its node look reached already, and the
    node's recovered arcs would be missing."""
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = shape_mix(g, 40, seed=poison)
    exp = [o.query(act, q) for q in qs]
    c = raks.Context(0, lanes=2, rec_caps=(1, 1, 1), poison=poison)
    try:
        c.load_graph(g, alpha=0.5)
        print(f"[poison {poison:#x}] single", flush=True)
        for q, e in zip(qs, exp):
            assert strip(c.query(q)) == e, ("single", q)
        print(f"[poison {poison:#x}] cohort", flush=True)
        for rep in range(2):
            for q, r, e in zip(qs, c.query_batch(qs), exp):
                assert strip(r) == e, ("cohort", rep, q)
    finally:
        c.close()
