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
