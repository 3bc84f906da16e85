"""The paper's multi-core CPU variant (Section 4.2.4) gives exactly the
reference implementation's results and counters, for any thread count and
for the scoring variants."""
from __future__ import annotations

import dataclasses

import pytest

import baselines
import oracle
import synth


@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("name", ["tiny", "tiny2", "small"])
def test_cpu_variant_matches_reference(name, threads):
    g = synth.make_graph(name)
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    cpu = baselines.CpuRaks(g)
    qs = synth.make_queries(g, name)[:24]
    qs += [dataclasses.replace(q, marginal=()) for q in qs[:3]]
    qs += [dataclasses.replace(q, score_mode=1, rerank=1) for q in qs[3:9]]
    qs += [dataclasses.replace(q, k=max(1, q.k // 3)) for q in qs[9:12]]
    for q in qs:
        assert cpu.query(act, q, threads) == o.query(act, q), (q, threads)


def test_cpu_variant_medium_sample():
    g = synth.make_graph("medium")
    o = oracle.Oracle(g, check=False)
    act = o.activation(g.abar, 0.5)
    cpu = baselines.CpuRaks(g)
    for q in synth.make_queries(g, "medium")[:2]:
        assert cpu.query(act, q, 8) == o.query(act, q)
