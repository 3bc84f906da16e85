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


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.8])
@pytest.mark.parametrize("name", ["tiny", "tiny2", "small"])
def test_cpu_variant_activation_matches_reference(name, alpha):
    """The variant's own activation levels (OpenMP, label runs per row) equal
    the reference's, per arc and per node."""
    g = synth.make_graph(name)
    o = oracle.Oracle(g)
    cpu = baselines.CpuRaks(g)
    for threads in (1, 4):
        assert (cpu.activation(g.abar, alpha, 0, threads) == o.activation(g.abar, alpha)).all()
        act_node_mode = o.activation(g.abar, alpha, oracle.MODE_NODE)[0]
        assert (cpu.activation(g.abar, alpha, 1, threads) == act_node_mode).all()


@pytest.mark.parametrize("block", [False, True])
def test_cpu_variant_exploration_matches_reference(block):
    """Exploration alone: the same counters as the reference's explore, for
    any thread count and level bound."""
    g = synth.make_graph("small")
    o = oracle.Oracle(g)
    act = o.activation(g.abar, 0.5)
    cpu = baselines.CpuRaks(g)
    for q in synth.make_queries(g, "small")[:6]:
        kws = list(q.central) + list(q.marginal)
        for L in (1, 3, 20):
            _, exp = o.explore(act, kws, block=block, max_level=L)
            for threads in (1, 5):
                got = cpu.explore(act, kws, block=block, max_level=L, threads=threads)
                for k in ("levels", "frontier", "e_arc", "e_alg", "gate_pass", "h_writes"):
                    assert got[k] == exp[k], (q, L, threads, k)
                assert got["end"] == exp["end"]
