"""CBDS-P on the GPU (dsg_cbds) against the CBDS-P oracle: the same core
number for every vertex, densest core (order, edges, vertices), eligible and
legitimate counts, result density and result set, on the hand-derived
examples, degenerate graphs, generated graphs with and without legitimate
vertices, and R-MAT scale 20."""
from __future__ import annotations

import json
from pathlib import Path

import numpy as np
import pytest

import oracle
from gpu_util import say, to_device
from paper_2103_00154_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = json.loads((Path(__file__).parent / "golden" / "cbds_examples.json").read_text())


def check(g):
    from paper_2103_00154_amd import dsg
    say(f"cbds {g.name} n={g.n} m={g.m}")
    rp, ci = to_device(g)
    r = dsg.cbds(rp, ci, m=g.m, core=True, trace=True)
    o = oracle.cbds(g)
    assert (r.num, r.den, r.core_num, r.core_den, r.K, r.n_legit) == (
        o.num, o.den, o.core_num, o.core_den, o.K, o.n_legit), (g.name, r, o)
    assert r.n_eligible == o.n_eligible
    if g.n:
        assert r.kmax == o.kmax
        assert np.array_equal(r.core.cpu().numpy(), o.core)
        assert np.array_equal(r.best.cpu().numpy(), o.best)
    # phase-1 levels never go down, and every level ends with a pass that
    # removes nothing (or with the pass that empties the graph)
    th = [t["thresh"] for t in r.trace]
    assert th == sorted(th)
    return r, o


@pytest.mark.parametrize("case", GOLDEN["cases"], ids=lambda c: c["name"])
def test_hand_derived_examples_on_gpu(case):
    r, _ = check(inputs.from_edges(case["n"], case["edges"]))
    assert (r.num, r.den, r.K) == (case["num"], case["den"], case["K"])


def test_degenerate_graphs():
    for g in (inputs.empty(1), inputs.empty(9), inputs.clique(2), inputs.clique(12),
              inputs.star(40), inputs.path(30), inputs.cycle(25), inputs.disjoint_cliques(11, 7)):
        check(g)


def test_empty_graph():
    import torch
    from paper_2103_00154_amd import dsg
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = dsg.cbds(rp, ci, m=0)
    assert (r.num, r.den, r.passes) == (0, 0, 0)


@pytest.mark.parametrize("seed", range(12))
def test_generated_graphs_with_legitimate_vertices(seed):
    g = inputs.rmat(10, 6, seed=seed, planted=(25, 0.6, seed + 100))
    check(g)


@pytest.mark.parametrize("gi", range(6))
def test_generated_families(gi):
    g = [inputs.erdos_renyi(20_000, 100_000, 1), inputs.chung_lu(50_000, 16, 2.2, 2),
         inputs.chung_lu(200_000, 24, 2.1, 3), inputs.rmat(16, 16, seed=4),
         inputs.rmat(14, 8, seed=5, planted=(200, 0.5, 6)),
         inputs.disjoint_cliques(300, 120)][gi]
    r, o = check(g)
    say(f"  K={r.K} kmax={r.kmax} passes={r.passes} legit={r.n_legit} eligible={r.n_eligible} "
        f"density {r.num}/{r.den}")


def test_rmat_scale20():
    g = inputs.rmat(20, 16, seed=0)
    r, o = check(g)
    say(f"  K={r.K} kmax={r.kmax} passes={r.passes} legit={r.n_legit} density {r.num}/{r.den}")
