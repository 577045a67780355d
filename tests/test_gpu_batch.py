"""Batched peeling on the GPU (dsg_batch_prepare / dsg_batch_run) against
the CPU oracle, graph by graph: the same passes, best pass, density, S~ and
removal pass of every vertex.  Covers mixed Erdos-Renyi / Chung-Lu batches,
the degenerate graphs, graphs whose vertex state does not fit in LDS (ids
beyond the LDS part and degrees above the 16-bit range), every launch shape,
per-graph eps, input-contract violations and replay of a captured HIP graph.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import say
from paper_2103_00154_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = [
    {"block": 256, "walk_items": 4}, {"block": 256, "walk_items": 8},
    {"block": 256, "walk_items": 16}, {"block": 512, "walk_items": 4},
    {"block": 512, "walk_items": 8}, {"block": 512, "walk_items": 16},
    {"block": 1024, "walk_items": 4}, {"block": 1024, "walk_items": 8},
    {"block": 512, "walk_items": 8, "blocks_per_cu": 2},
    {"block": 256, "walk_items": 8, "blocks_per_cu": 4},
    # a few hundred vertices of LDS state: almost every vertex in device memory
    {"block": 256, "walk_items": 16, "blocks_per_cu": 8},
    {"block": 1024, "walk_items": 4, "grid": 3},
]


def _eps_of(eps, i):
    return eps[i] if isinstance(eps[0], (tuple, list)) else eps


def run_batch(b, eps=(1, 10), launch=None):
    import torch
    from paper_2103_00154_amd import dsg
    rp = torch.from_numpy(b.row_ptr).cuda()
    ci = torch.from_numpy(b.col_idx).cuda()
    tab, count = dsg.batch_table(b.n, b.m, b.rp_off, b.ci_off, b.out_off, eps)
    plan = dsg.Batch(tab, count, len(b.row_ptr), len(b.col_idx), b.out_len, launch=launch)
    best = torch.full((max(b.out_len, 1),), -7, dtype=torch.int32, device="cuda")
    rem = torch.full((max(b.out_len, 1),), -7, dtype=torch.int32, device="cuda")
    res = plan.run(rp, ci, best_ids=best, removed_at=rem)
    torch.cuda.synchronize()
    return dsg.Batch.results(res)[:count], best.cpu().numpy(), rem.cpu().numpy(), plan


def oracle_all(b, eps=(1, 10)):
    return [oracle.peel_graph(b.graph(i), *_eps_of(eps, i), trace=False) for i in range(b.count)]


def check_batch(b, eps=(1, 10), launch=None, want=None):
    say(f"batch of {b.count} graphs, {b.out_len} vertices, {int(b.m.sum())} edges, "
        f"launch {launch}")
    results, best, rem, plan = run_batch(b, eps, launch)
    want = want if want is not None else oracle_all(b, eps)
    for i in range(b.count):
        o, r, n, a = want[i], results[i], int(b.n[i]), int(b.out_off[i])
        assert r["status"] == 0, (i, r)
        assert (r["passes"], r["best_pass"], r["num"], r["den"]) == (
            o.passes, o.best_pass, o.num, o.den), (i, r, (o.passes, o.best_pass, o.num, o.den))
        assert r["best_size"] == len(o.best), i
        assert np.array_equal(best[a:a + r["best_size"]], o.best), i
        assert np.array_equal(rem[a:a + n], o.removed_at[:n]), i
    return plan, want


def test_mixed_small_batch_default_shape():
    b = inputs.make_batch(inputs.batch_specs(96, seed=3, n_range=(100, 20_000)))
    plan, _ = check_batch(b)
    say(f"shape {plan.shape}")


def test_degenerate_graphs():
    gs = [inputs.empty(0), inputs.empty(1), inputs.empty(7), inputs.clique(2),
          inputs.from_edges(5, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (0, 4)]),
          inputs.from_edges(6, [(1, 4), (1, 5), (3, 4)]),
          inputs.from_edges(4, [(0, 2), (0, 3), (1, 3), (2, 3)]),
          inputs.path(3), inputs.star(50), inputs.cycle(40), inputs.clique(30),
          inputs.disjoint_cliques(12, 5), inputs.empty(0),
          inputs.from_edges(8, [(i, j) for i in range(5) for j in range(i + 1, 5)]
                            + [(4, 5), (5, 6), (6, 7)])]
    b = inputs.concat(gs)
    for eps in ((0, 1), (1, 10), (1, 1), (7, 3)):
        check_batch(b, eps)


def test_per_graph_eps():
    b = inputs.make_batch(inputs.batch_specs(40, seed=5, n_range=(100, 5000)))
    choices = [(1, 100), (1, 10), (1, 2), (0, 1), (3, 1)]
    eps = [choices[i % len(choices)] for i in range(b.count)]
    check_batch(b, eps)


def test_graph_larger_than_lds_with_hub_degrees_above_16_bits():
    # n beyond every LDS capacity; Chung-Lu exponent 2.1 gives hubs whose
    # degree exceeds the 16-bit range of the LDS state
    big = inputs.chung_lu(200_000, 64, 2.1, seed=11)
    deg = big.degrees()
    assert deg.max() >= 0xFE00 and big.n > 80_000
    gs = [big, inputs.chung_lu(3000, 20, 2.5, seed=12), inputs.erdos_renyi(90_000, 400_000, 13)]
    b = inputs.concat(gs)
    want = oracle_all(b)
    for launch in (None, {"block": 512, "walk_items": 16, "blocks_per_cu": 2},
                   {"block": 256, "walk_items": 16, "blocks_per_cu": 8}):
        check_batch(b, launch=launch, want=want)


def test_every_launch_shape_gives_the_same_results():
    b = inputs.make_batch(inputs.batch_specs(48, seed=7, n_range=(100, 60_000)))
    want = oracle_all(b)
    for launch in SHAPES:
        plan, _ = check_batch(b, launch=launch, want=want)
        say(f"ok {plan.shape}")


def test_contract_violations_are_reported_per_graph():
    import torch
    from paper_2103_00154_amd import dsg
    good = inputs.erdos_renyi(300, 900, 1)
    b = inputs.concat([good, good, good, good])
    # graph 1: row_ptr[n] != 2m; graph 2: decreasing row offsets;
    # graph 3: a neighbour id outside 0..n-1
    a1, a2 = int(b.rp_off[1]), int(b.rp_off[2])
    b.row_ptr[a1 + 300] -= 2
    k = int(np.flatnonzero(np.diff(good.row_ptr[1:]) > 0)[0]) + 1  # rows k, k+1 differ
    b.row_ptr[a2 + k], b.row_ptr[a2 + k + 1] = b.row_ptr[a2 + k + 1], b.row_ptr[a2 + k]
    # (in the row of a vertex whose row is walked: it fails in pass 1 with
    # a neighbour left, and pass 1 leaves survivors)
    o = oracle.peel_graph(good, 1, 10, trace=False)
    assert o.passes > 1
    v = int(np.flatnonzero((o.removed_at == 1) & (good.degrees() > 0))[0])
    b.col_idx[int(b.ci_off[3]) + int(good.row_ptr[v])] = 5000
    results, best, rem, _ = run_batch(b)
    assert results[0]["status"] == 0
    assert (results[0]["num"], results[0]["den"], results[0]["passes"]) == (o.num, o.den, o.passes)
    assert [r["status"] for r in results[1:]] == [dsg.DSG_EINVAL] * 3


@pytest.mark.parametrize("large", [False, True], ids=["16-bit", "8-bit"])
def test_hip_graph_capture_and_replay(large):
    import torch
    from paper_2103_00154_amd import dsg
    b = inputs.make_batch(inputs.batch_specs(64, seed=9, n_range=(100, 30_000)))
    if large:
        # a graph above the 16-bit LDS states: the plan takes 8-bit states
        b = inputs.concat([b.graph(i) for i in range(b.count)] +
                          [inputs.chung_lu(95_000, 40, 2.1, seed=10)])
    want = oracle_all(b)
    rp = torch.from_numpy(b.row_ptr).cuda()
    ci = torch.from_numpy(b.col_idx).cuda()
    tab, count = dsg.batch_table(b.n, b.m, b.rp_off, b.ci_off, b.out_off, (1, 10))
    plan = dsg.Batch(tab, count, len(b.row_ptr), len(b.col_idx), b.out_len)
    assert plan.shape["state_bits"] == (8 if large else 16)
    best = torch.full((b.out_len,), -1, dtype=torch.int32, device="cuda")
    res = torch.zeros((count, dsg.RESULT_WORDS), dtype=torch.int64, device="cuda")
    plan.run(rp, ci, best_ids=best, results=res)  # eager run before capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(rp, ci, best_ids=best, results=res)
    other = torch.zeros_like(res)
    for rep in range(3):
        best.fill_(-1)
        res.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = dsg.Batch.results(res)
        h_best = best.cpu().numpy()
        for i in range(count):
            o, r, a = want[i], got[i], int(b.out_off[i])
            assert (r["status"], r["passes"], r["num"], r["den"], r["best_size"]) == (
                0, o.passes, o.num, o.den, len(o.best)), (rep, i)
            assert np.array_equal(h_best[a:a + len(o.best)], o.best), (rep, i)
        # eager work on the same plan between replays
        plan.run(rp, ci, results=other)
        torch.cuda.synchronize()
        assert dsg.Batch.results(other) == [dict(g, best_size=0) for g in got]
        say(f"replay {rep} ok")


def _with_clique(n_extra, extra_edges, k=60):
    """A k-clique on ids 0..k-1 plus `extra_edges` on ids k..k+n_extra-1."""
    core = [(i, j) for i in range(k) for j in range(i + 1, k)]
    return inputs.from_edges(k + n_extra, core + [(k + a, k + b) for a, b in extra_edges])


def test_wave_tiles_over_many_short_rows():
    # the clique survives the first pass while the pendant structures fail
    # with rows of length 1, so one wave tile spans hundreds of walked rows:
    # more than the 256 whose starts and bases are loaded one tile ahead
    matching = _with_clique(20_000, [(2 * i, 2 * i + 1) for i in range(10_000)])
    stars = _with_clique(40_000, [(4 * i, 4 * i + j) for i in range(10_000) for j in (1, 2, 3)])
    paths = _with_clique(30_000, [(i, i + 1) for i in range(29_999) if i % 3 != 2])
    b = inputs.concat([matching, stars, paths, inputs.clique(40)])
    want = oracle_all(b)
    assert all(o.passes >= 2 for o in want[:3])
    for launch in (None, {"block": 256, "walk_items": 16}, {"block": 1024, "walk_items": 4},
                   {"block": 512, "walk_items": 4}):
        check_batch(b, launch=launch, want=want)


def test_eight_bit_states_with_hubs_and_a_full_hash_table():
    # the largest graph exceeds the 16-bit states, so the plan takes 8-bit
    # states: degrees of 240 and more go to the LDS hash table, and the dense
    # graph has far more of them than the table's 4096 slots (the rest keep
    # their degree in device memory)
    from paper_2103_00154_amd import dsg
    small = inputs.make_batch(inputs.batch_specs(8, seed=3, n_range=(100, 2000)))
    tab, _ = dsg.batch_table(small.n, small.m, small.rp_off, small.ci_off, small.out_off, (1, 10))
    assert dsg.Batch(tab, small.count, len(small.row_ptr), len(small.col_idx),
                     small.out_len).shape["state_bits"] == 16
    dense = inputs.erdos_renyi(80_000, 10_400_000, 31)
    assert (dense.degrees() >= 240).sum() > 4096
    hubs = inputs.chung_lu(99_000, 48, 2.1, seed=32)
    gs = [dense, hubs, inputs.erdos_renyi(3000, 9000, 33), inputs.empty(5),
          inputs.chung_lu(20_000, 30, 2.3, seed=34)]
    b = inputs.concat(gs)
    want = oracle_all(b)
    plan, _ = check_batch(b, (0, 1))
    assert plan.shape["state_bits"] == 8 and plan.shape["lds_vertices"] >= 99_000, plan.shape
    # every shape with one workgroup per CU holds 8-bit states for more
    # vertices than 16-bit ones
    for launch in SHAPES:
        if launch.get("blocks_per_cu", 1) != 1:
            continue
        plan, _ = check_batch(b, launch=launch, want=want)
        assert plan.shape["state_bits"] == 8, plan.shape
        say(f"8-bit plan: {plan.shape}")
