"""The exact densest subgraph on the GPU (dsg_exact_density: Goldberg's
construction, Section 2, with a device push-relabel flow in Dinkelbach's
iteration) against the oracle: rho* as a fraction equals
oracle.exact.densest_goldberg, and the set equals the largest densest
subgraph of oracle.exact.densest_maximal (unique), on brute-force-checked
small graphs, the four graphs of the eps-sweep guarantee test and generated
graphs of 10^4 to 2.6 * 10^5 vertices.  The peel's (2 + 2 eps) guarantee is then
checked against the GPU's rho*.
"""
from __future__ import annotations

import itertools
import random

import numpy as np
import pytest

import oracle
from gpu_util import say, to_device
from oracle import exact
from paper_2103_00154_amd import inputs

pytestmark = pytest.mark.gpu


def _edges(g):
    return [tuple(map(int, e)) for e in g.edges()]


def run(g):
    from paper_2103_00154_amd import dsg
    rp, ci = to_device(g)
    return dsg.exact_density(rp, ci, m=g.m)


def check(g, goldberg=True):
    say(f"case {g.name} n={g.n} m={g.m}")
    r = run(g)
    e, s, mask = exact.densest_maximal(g.n, g.edges())
    assert (r.num, r.den) == (e, s), ((r.num, r.den), (e, s))
    assert np.array_equal(r.best.cpu().numpy(), np.flatnonzero(mask))
    if goldberg:
        eg, sg, _ = exact.densest_goldberg(g.n, g.edges())
        assert r.num * sg == eg * r.den
    say(f"  rho* = {r.num}/{r.den} = {r.density:.4f}, {r.flows} flows, {r.relabels} relabels")
    return r


def test_small_graphs_against_bruteforce():
    rnd = random.Random(41)
    for i in range(80):
        n = rnd.randint(1, 11)
        pairs = list(itertools.combinations(range(n), 2))
        p = rnd.choice([0.15, 0.3, 0.5, 0.9])
        g = inputs.from_edges(n, [x for x in pairs if rnd.random() < p])
        r = run(g)
        e, s, mask = exact.densest_maximal(n, _edges(g))
        eb, sb, _ = exact.densest_bruteforce(n, _edges(g))
        assert (r.num, r.den) == (e, s) and r.num * sb == eb * r.den, (i, r, e, s)
        assert np.array_equal(r.best.cpu().numpy(), np.flatnonzero(mask)), i


def test_closed_forms():
    r = check(inputs.disjoint_cliques(30, 30))  # both cliques are densest: their union
    assert (r.num, r.den) == (2 * 435, 60)
    r = check(inputs.disjoint_cliques(30, 12))
    assert (r.num, r.den) == (435, 30)
    r = check(inputs.empty(7), goldberg=False)  # no edge: every vertex, density 0
    assert (r.num, r.den) == (0, 7)
    r = check(inputs.star(200))
    assert (r.num, r.den) == (199, 200)
    check(inputs.path(50))
    check(inputs.cycle(40))
    check(inputs.clique(64))


def test_empty_vertex_set():
    import torch
    from paper_2103_00154_amd import dsg
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = dsg.exact_density(rp, ci, m=0)
    assert (r.num, r.den, r.flows) == (0, 0, 0)


@pytest.mark.parametrize("gi", range(4))
def test_sweep_graphs(gi):
    g = [inputs.chung_lu(1500, 12, 2.2, seed=3), inputs.erdos_renyi(1200, 9000, 4),
         inputs.rmat(11, 8, seed=6), inputs.rmat(11, 16, seed=7, planted=(40, 0.6, 8))][gi]
    check(g)


@pytest.mark.parametrize("gi", range(7))
def test_graphs_of_ten_thousand_to_a_quarter_million_vertices(gi):
    g = [inputs.erdos_renyi(10_000, 50_000, 0), inputs.chung_lu(50_000, 16, 2.2, 2),
         inputs.chung_lu(100_000, 24, 2.5, 5), inputs.rmat(16, 16, seed=4),
         inputs.rmat(14, 8, seed=8, planted=(300, 0.4, 9)),
         inputs.erdos_renyi(100_000, 1_000_000, 3), inputs.rmat(18, 16, seed=0)][gi]
    check(g, goldberg=False)


def test_peel_guarantee_against_the_gpu_optimum():
    from paper_2103_00154_amd import dsg
    for g in (inputs.rmat(16, 16, seed=4), inputs.chung_lu(50_000, 16, 2.2, 2)):
        rp, ci = to_device(g)
        x = dsg.exact_density(rp, ci, extract=False)
        for num, den in ((0, 1), (1, 100), (1, 10), (1, 1), (5, 1)):
            p = dsg.peel(rp, ci, (num, den))
            o = oracle.peel_graph(g, num, den, trace=False)
            assert (p.num, p.den) == (o.num, o.den)
            assert 2 * (num + den) * p.num * x.den >= den * x.num * p.den
            assert p.num * x.den <= x.num * p.den  # no set beats rho*
            say(f"{g.name} eps {num}/{den}: rho(S~)/rho* = {p.num * x.den / (p.den * x.num):.4f}")
