"""Seeded input generators: determinism and CSR validity (no GPU)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2103_00154_amd import inputs


def _valid(g):
    assert g.row_ptr.dtype == np.int32 and g.col_idx.dtype == np.int32
    assert len(g.row_ptr) == g.n + 1 and g.row_ptr[0] == 0 and g.row_ptr[-1] == 2 * g.m
    assert oracle.check_csr(g.row_ptr, g.col_idx, g.n) == 0


def test_er_config_small():
    g = inputs.erdos_renyi(10000, 50000, 0)
    _valid(g)
    assert (g.n, g.m) == (10000, 50000)


def test_generators_are_deterministic():
    for make in (lambda: inputs.rmat(12, 8, seed=5),
                 lambda: inputs.chung_lu(5000, 16, 2.5, 2),
                 lambda: inputs.erdos_renyi(3000, 9000, 4),
                 lambda: inputs.rmat(11, 4, seed=1, planted=(50, 0.5, 3))):
        a, b = make(), make()
        assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col_idx, b.col_idx)
        _valid(a)


def test_seed_changes_graph():
    a, b = inputs.rmat(10, 8, seed=0), inputs.rmat(10, 8, seed=1)
    assert not np.array_equal(a.col_idx[:100], b.col_idx[:100])


def test_rmat_is_skewed_towards_low_ids():
    g = inputs.rmat(14, 16, seed=0)
    deg = g.degrees()
    assert deg[:64].mean() > 20 * deg.mean()
    assert g.m < 16 * g.n  # loops and repeats removed


def test_planted_block_is_present():
    g = inputs.rmat(12, 4, seed=0, planted=(100, 0.5, 1))
    ids = g.meta["planted_ids"]
    assert len(set(ids.tolist())) == 100
    e = g.edges()
    inside = np.isin(e[:, 0], ids) & np.isin(e[:, 1], ids)
    # G(100, 1/2) has 2475 edges in expectation; sd ~ 35
    assert 2200 < int(inside.sum()) < 2800


def test_chung_lu_power_law_tail():
    g = inputs.chung_lu(20000, 16, 2.1, 0)
    deg = g.degrees()
    assert deg.max() > 50 * np.median(deg)


def test_from_edges_and_relabel():
    g = inputs.from_edges(5, [(0, 1), (1, 0), (3, 4)])
    assert g.m == 2
    _valid(g)
    with pytest.raises(ValueError):
        inputs.from_edges(3, [(1, 1)])
    h = inputs.relabel(g, np.array([4, 3, 2, 1, 0]))
    assert sorted(map(tuple, h.edges().tolist())) == [(0, 1), (3, 4)]


def test_counter_rng_fixed_values():
    # splitmix64-based counter stream: fixed values guard against accidental
    # changes of the input recipe
    vals = [inputs.draw_for_test(0, 1, i) for i in range(3)]
    assert len(set(vals)) == 3
    assert vals == [inputs.draw_for_test(0, 1, i) for i in range(3)]


# ---------------------------------------------------------------- batches

def test_batch_graphs_equal_the_single_generators():
    specs = inputs.batch_specs(24, seed=2, n_range=(100, 3000))
    b = inputs.make_batch(specs)
    assert b.count == 24 and b.out_len == sum(s.n for s in specs)
    assert {s.kind for s in specs} == {inputs.KIND_ER, inputs.KIND_CHUNG_LU}
    for i, s in enumerate(specs):
        g = b.graph(i)
        if s.kind == inputs.KIND_ER:
            ref = inputs.erdos_renyi(s.n, s.size, s.seed)
        else:
            ref = inputs.chung_lu(s.n, s.avg_deg, s.gamma, s.seed)
        assert g.n == ref.n and g.m == ref.m
        assert np.array_equal(g.row_ptr, ref.row_ptr)
        assert np.array_equal(g.col_idx, ref.col_idx)


def test_batch_specs_follow_the_recipe():
    specs = inputs.batch_specs(400, seed=0)
    n = np.array([s.n for s in specs])
    assert n.min() >= 100 and n.max() <= 100_000
    # log-uniform: about half of the graphs below the geometric midpoint
    assert 150 < np.count_nonzero(n < np.sqrt(100 * 100_000)) < 250
    d = np.array([s.avg_deg for s in specs])
    assert d.min() >= 4 and d.max() <= 64
    g = np.array([s.gamma for s in specs if s.kind == inputs.KIND_CHUNG_LU])
    assert len(g) == 200 and g.min() >= 2.1 and g.max() <= 2.8
    assert specs[5].seed == 5 and inputs.batch_specs(3, seed=1)[2].seed == (1 << 32) + 2


def test_concat_round_trips_and_offsets_are_disjoint():
    gs = [inputs.empty(0), inputs.clique(5), inputs.path(7), inputs.empty(3), inputs.star(9)]
    b = inputs.concat(gs)
    for i, g in enumerate(gs):
        h = b.graph(i)
        assert (h.n, h.m) == (g.n, g.m)
        assert np.array_equal(h.row_ptr, g.row_ptr)
        assert np.array_equal(h.col_idx, g.col_idx[:2 * g.m])
    ends = b.out_off + b.n
    assert np.all(ends[:-1] <= b.out_off[1:]) and ends[-1] == b.out_len
