"""Pins of the CBDS-P oracle (Section 3.2, Algorithm 2): the C oracle against
the definition-level restatement, hand-derived examples, closed forms, and
the approximation facts the paper relies on (the densest k-core is within a
factor 2 of the densest subgraph; adding legitimate vertices only raises
the density)."""
from __future__ import annotations

import itertools
import json
import random
from fractions import Fraction
from pathlib import Path

import numpy as np
import pytest

import oracle
from oracle import exact
from oracle.cbds_literal import cbds_literal
from paper_2103_00154_amd import inputs

GOLDEN = json.loads((Path(__file__).parent / "golden" / "cbds_examples.json").read_text())


def _edges(g):
    return [tuple(map(int, e)) for e in g.edges()]


def _same(g):
    c = oracle.cbds(g)
    lit = cbds_literal(g.n, _edges(g))
    assert (c.num, c.den) == (lit["num"], lit["den"]), g.name
    assert (c.num, c.den) == lit["claimed"], g.name
    assert c.K == lit["K"] and c.core.tolist() == lit["core"]
    assert c.best.tolist() == lit["best"]
    assert c.n_legit == len(lit["legit"])
    assert (c.core_num, c.core_den) == (lit["core_num"], lit["core_den"])
    return c


@pytest.mark.parametrize("case", GOLDEN["cases"], ids=lambda c: c["name"])
def test_hand_derived_examples(case):
    g = inputs.from_edges(case["n"], case["edges"])
    c = _same(g)
    assert c.core.tolist() == case["core"]
    assert (c.K, c.core_num, c.core_den, c.num, c.den) == (
        case["K"], case["core_num"], case["core_den"], case["num"], case["den"])
    assert c.best.tolist() == case["best"]
    assert c.n_legit == len(case["legit"])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_every_graph_up_to_five_vertices(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        g = inputs.from_edges(n, [p for i, p in enumerate(pairs) if mask >> i & 1])
        _same(g)


@pytest.mark.parametrize("seed", range(60))
def test_random_graphs_against_the_definitions(seed):
    rnd = random.Random(seed)
    n = rnd.randint(6, 40)
    g = inputs.random_small(n, rnd.choice([0.05, 0.1, 0.2, 0.4, 0.7]), seed)
    _same(g)


def test_closed_forms():
    for k in (2, 5, 9):
        c = oracle.cbds(inputs.clique(k))
        assert set(c.core.tolist()) == {k - 1} and (c.num, c.den) == (k * (k - 1) // 2, k)
    c = oracle.cbds(inputs.star(12))
    assert set(c.core.tolist()) == {1} and (c.num, c.den, c.K) == (11, 12, 0)
    c = oracle.cbds(inputs.cycle(15))
    assert set(c.core.tolist()) == {2} and (c.num, c.den) == (15, 15)
    c = oracle.cbds(inputs.path(9))
    assert set(c.core.tolist()) == {1}
    c = oracle.cbds(inputs.disjoint_cliques(9, 6))
    assert c.core.tolist() == [8] * 9 + [5] * 6
    assert (c.num, c.den, c.n_legit) == (36, 9, 0)
    c = oracle.cbds(inputs.empty(5))
    assert (c.num, c.den, c.K, c.kmax) == (0, 5, 0, 0)
    c = oracle.cbds(inputs.empty(0))
    assert (c.num, c.den) == (0, 0)


def _graphs():
    yield inputs.erdos_renyi(300, 1500, 0)
    yield inputs.rmat(9, 8, seed=2)
    yield inputs.chung_lu(500, 10, 2.2, 3)
    yield inputs.rmat(10, 4, seed=4, planted=(30, 0.7, 5))
    yield inputs.chung_lu(800, 6, 2.5, 6)


@pytest.mark.parametrize("gi", range(5))
def test_approximation_facts(gi):
    g = list(_graphs())[gi]
    c = oracle.cbds(g)
    e_star, s_star, _ = exact.densest_goldberg(g.n, g.edges())
    # the densest core is within a factor 2 of rho* (Section 2)
    assert 2 * c.core_num * s_star >= e_star * c.core_den
    # legitimate vertices only raise the density, never above rho*
    assert c.num * c.core_den >= c.core_num * c.den
    if c.n_legit:
        assert c.num * c.core_den > c.core_num * c.den
    assert c.num * s_star <= e_star * c.den
    # the reported counts are those of the returned set
    ids = set(c.best.tolist())
    assert c.den == len(ids)
    assert c.num == sum(1 for u, v in _edges(g) if u in ids and v in ids)


def test_core_numbers_match_the_definition_on_generated_graphs():
    for g in list(_graphs())[:3]:
        c = oracle.cbds(g)
        lit = cbds_literal(g.n, _edges(g))
        assert c.core.tolist() == lit["core"]


def test_printed_label_reading_misreports_the_density():
    # recording the level just peeled as the core order (the printed update)
    # lets core-number-K vertices outside the densest core count as inside:
    # the reported density then differs from the returned set's density
    case = GOLDEN["cases"][0]
    lit = cbds_literal(case["n"], [tuple(e) for e in case["edges"]], printed_label=True)
    assert lit["claimed"] != (lit["num"], lit["den"])
    ours = cbds_literal(case["n"], [tuple(e) for e in case["edges"]])
    assert ours["claimed"] == (ours["num"], ours["den"])


def test_relabelling_permutes_the_result():
    g = inputs.chung_lu(400, 8, 2.3, 9)
    perm = np.random.default_rng(1).permutation(g.n)
    h = inputs.relabel(g, perm)
    a, b = oracle.cbds(g), oracle.cbds(h)
    assert (a.num, a.den, a.K, a.n_legit) == (b.num, b.den, b.K, b.n_legit)
    assert sorted(perm[a.best].tolist()) == b.best.tolist()
    assert np.array_equal(a.core, b.core[perm])


def test_legit_extension_happens_on_generated_graphs():
    # at least one generated case exercises phase 2 (otherwise the pins above
    # would only cover the densest-core phase)
    found = 0
    for seed in range(40):
        g = inputs.rmat(10, 6, seed=seed, planted=(25, 0.6, seed + 100))
        c = oracle.cbds(g)
        if c.n_legit:
            _same(g) if g.n <= 1024 else None
            found += 1
    assert found > 0
