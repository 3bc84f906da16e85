"""Scoring variants on the GPU (Section 3.3): the multiplicative combination
S^c * S^m and the re-ranking of equal scores by the sum of the results' arc
levels (with the strict Theorem 4 it needs), alone and together, against the
reference implementation: results, order, weight sums, status and counters
bit for bit."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

MODES = [(1, 0), (0, 1), (1, 1)]
IDS = ["mult", "rerank", "mult-rerank"]


def strip(r):
    r = dict(r)
    for k in ("device_ms", "host_ms", "queue_ms"):
        r.pop(k, None)
    return r


@pytest.fixture(scope="module")
def raks():
    import paper_2001_06770_amd as raks
    return raks


@pytest.mark.parametrize("mode", MODES, ids=IDS)
@pytest.mark.parametrize("name", ["tiny2", "small"])
def test_scoring_variants_match_reference(raks, name, mode):
    g = synth.make_graph(name)
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = [dataclasses.replace(q, score_mode=mode[0], rerank=mode[1])
          for q in synth.make_queries(g, name)[:24]]
    # without marginal keywords too, and a few with w > k
    qs += [dataclasses.replace(q, marginal=(), score_mode=mode[0], rerank=mode[1])
           for q in qs[:4]]
    qs += [dataclasses.replace(q, k=max(1, q.k // 2), score_mode=mode[0], rerank=mode[1])
           for q in qs[4:8]]
    c = raks.Context(0, lanes=2)
    try:
        c.load_graph(g, alpha=0.5)
        exp = [o.query(act, q) for q in qs]
        for q, e in zip(qs, exp):
            assert strip(c.query(q)) == e, q
        for q, r, e in zip(qs, c.query_batch(qs), exp):
            assert strip(r) == e, q
    finally:
        c.close()


def test_scoring_variants_medium(raks):
    g = synth.make_graph("medium")
    o = oracle.Oracle(g, check=False)
    act = o.activation(g.abar, 0.5)
    qs = synth.make_queries(g, "medium")[:3]
    c = raks.Context(0)
    try:
        c.load_graph(g, alpha=0.5)
        for mode in MODES:
            for q in qs:
                qm = dataclasses.replace(q, score_mode=mode[0], rerank=mode[1])
                assert strip(c.query(qm)) == o.query(act, qm), qm
    finally:
        c.close()


def test_rerank_through_bitmap_path(raks):
    """Re-ranking after the bitmap merge of large results (forced with a tiny
    threshold): the arc-level sums come from the bitmap path then."""
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    qs = [dataclasses.replace(q, rerank=1) for q in synth.make_queries(g, "small")[:12]]
    c = raks.Context(0, big_list=8)
    try:
        c.load_graph(g, alpha=0.5)
        for q in qs:
            assert strip(c.query(q)) == o.query(act, q), q
    finally:
        c.close()


def test_invalid_scoring_options(raks):
    g = synth.make_graph("tiny")
    c = raks.Context(0)
    try:
        c.load_graph(g, alpha=0.5)
        q = synth.make_queries(g, "tiny")[0]
        for bad in (dict(score_mode=2), dict(rerank=-1)):
            with pytest.raises(raks.RaksError) as e:
                c.query(dataclasses.replace(q, **bad))
            assert e.value.code == -1
    finally:
        c.close()
