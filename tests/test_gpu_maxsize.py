"""A graph just below the int32 limit of adjacency entries (2m = 2,147,481,600
of at most 2^31 - 1), built on the GPU, with a result known in closed form.

The graph: n 64-cliques' worth of vertices (ids 0..n-1, cliques of 64
consecutive ids) and n 32-cliques' worth (ids n..2n-1), plus one bridge edge
from vertex j to vertex n + j.  Degrees are 64 and 32, |E| = 48n, rho = 24.
With eps = 1/10 the first threshold is floor(2 * 1.1 * 24) = 52: every
32-clique vertex fails, each bridge is a cross entry (one degree-update
record per 64-clique vertex), the 31 clique entries of each failed row are
intra.  What is left is the 64-cliques, |E| = 63n/2, density 31.5 > 24, the
best graph; the second threshold, floor(2.2 * 31.5) = 69, removes the rest.
A small instance pins this closed form against the oracle.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import say
from paper_2103_00154_amd import inputs

pytestmark = pytest.mark.gpu

N_MAX = 22_369_600  # 96 * N_MAX = 2,147,481,600 adjacency entries


def bridged_cliques(n_side: int, device):
    """row_ptr, col_idx (torch int32) of the graph above; n_side % 64 == 0."""
    import torch
    i32 = torch.int32
    assert n_side % 64 == 0 and 96 * n_side < 2**31
    v = torch.arange(n_side, dtype=i32, device=device).view(-1, 1)
    k = torch.arange(63, dtype=i32, device=device).view(1, -1)
    off = v % 64
    big = (v - off) + k + (k >= off).to(i32)            # clique mates, ascending
    big = torch.cat([big, v + n_side], dim=1)           # then the bridge
    del k, off
    k = torch.arange(31, dtype=i32, device=device).view(1, -1)
    off = v % 32
    small = n_side + (v - off) + k + (k >= off).to(i32)
    small = torch.cat([v, small], dim=1)                # the bridge first
    del k, off
    ci = torch.cat([big.reshape(-1), small.reshape(-1)])
    del big, small, v
    i64 = torch.int64
    rp = torch.cat([torch.arange(n_side + 1, dtype=i64, device=device) * 64,
                    64 * n_side + 32 * torch.arange(1, n_side + 1, dtype=i64, device=device)])
    return rp.to(i32), ci


def expected(n_side: int, eps):
    """(passes, best_pass, num, den, removal pass of the 64-clique part and
    of the 32-clique part) for eps in {1/10, 0}, or for eps = 1 (threshold
    96: everything fails in pass 1, the whole graph is the best)."""
    if tuple(eps) == (1, 1):
        return 1, 0, 48 * n_side, 2 * n_side, 1, 1
    return 2, 1, 63 * n_side // 2, n_side, 2, 1


def check_closed_form(r, n_side, eps):
    passes, best_pass, num, den, rem_big, rem_small = expected(n_side, eps)
    assert (r.passes, r.best_pass, r.num, r.den) == (passes, best_pass, num, den)
    rem = r.removed_at
    assert bool((rem[:n_side] == rem_big).all()) and bool((rem[n_side:] == rem_small).all())
    if best_pass == 1:
        import torch
        ids = torch.arange(n_side, dtype=torch.int32, device=r.best.device)
        assert r.best.numel() == n_side and bool((r.best == ids).all())
        t = r.trace[0]
        assert (t["s_in"], t["removed"], t["cross"], t["intra"], t["s_out"], t["e_out"]) == (
            2 * n_side, n_side, n_side, 31 * n_side, n_side, 63 * n_side // 2)
    else:
        assert r.best.numel() == 2 * n_side


@pytest.mark.parametrize("eps", [(1, 10), (0, 1), (1, 1)])
def test_closed_form_against_oracle_small(eps):
    import torch
    from paper_2103_00154_amd import dsg
    n_side = 64 * 40
    rp, ci = bridged_cliques(n_side, "cpu")
    g = inputs.Graph(2 * n_side, ci.numel() // 2, rp.numpy(), ci.numpy(), name="bridged")
    o = oracle.peel_graph(g, *eps)
    passes, best_pass, num, den, rem_big, rem_small = expected(n_side, eps)
    assert (o.passes, o.best_pass, o.num, o.den) == (passes, best_pass, num, den)
    assert np.all(o.removed_at[:n_side] == rem_big) and np.all(o.removed_at[n_side:] == rem_small)
    r = dsg.peel(rp.cuda(), ci.cuda(), eps, removed_at=True, trace=True)
    check_closed_form(r, n_side, eps)
    assert np.array_equal(r.best.cpu().numpy(), o.best)
    del r
    torch.cuda.empty_cache()


def test_adjacency_entries_just_below_int32_limit():
    import torch
    from paper_2103_00154_amd import dsg
    say(f"building bridged cliques on the GPU: n = {2 * N_MAX}, 2m = {96 * N_MAX}")
    rp, ci = bridged_cliques(N_MAX, "cuda")
    torch.cuda.synchronize()
    assert ci.numel() == 96 * N_MAX and ci.numel() <= 2**31 - 1
    assert int(rp[-1]) == ci.numel()
    say("validating the CSR on the device")
    assert dsg.validate_csr(rp, ci) == 0
    ws = dsg.alloc_workspace(2 * N_MAX, ci.numel() // 2)
    for eps in ((1, 10), (0, 1), (1, 1)):
        say(f"peel eps = {eps[0]}/{eps[1]}")
        r = dsg.peel(rp, ci, eps, removed_at=True, trace=True, workspace=ws)
        check_closed_form(r, N_MAX, eps)
        del r
    del rp, ci, ws
    torch.cuda.empty_cache()


def test_id_keyed_pass_with_the_most_buckets():
    # n = 2^25, the most vertices whose passes may key their degree records
    # by neighbour id (1024 buckets of 32768 ids), and 2m = 1.61 G: pass 1
    # walks 537 M entries and leaves 16.8 M survivors, so by default it takes
    # the id-keyed walk with about 32,800 record groups
    import torch
    from paper_2103_00154_amd import dsg
    n_side = 1 << 24
    say(f"building bridged cliques on the GPU: n = {2 * n_side}, 2m = {96 * n_side}")
    rp, ci = bridged_cliques(n_side, "cuda")
    ws = dsg.alloc_workspace(2 * n_side, ci.numel() // 2)
    for eps in ((1, 10), (0, 1), (1, 1)):
        say(f"peel eps = {eps[0]}/{eps[1]}")
        r = dsg.peel(rp, ci, eps, removed_at=True, trace=True, workspace=ws)
        check_closed_form(r, n_side, eps)
        if tuple(eps) != (1, 1):
            t = r.trace[0]
            assert t["s_out"] > 65536 and t["walked"] >= 1 << 25, t
        del r
    del rp, ci, ws
    torch.cuda.empty_cache()


def test_batch_with_col_idx_offsets_beyond_int32():
    # three bridged-clique graphs of 768 M adjacency entries each, back to
    # back: the third one starts past entry 2^31 of the concatenated arrays,
    # so only the 64-bit per-graph offsets reach it
    import torch
    from paper_2103_00154_amd import dsg
    n_side = 8_000_000
    rp, ci = bridged_cliques(n_side, "cuda")
    count, n, e = 3, 2 * n_side, ci.numel()
    rp_all = rp.repeat(count)
    ci_all = ci.repeat(count)
    del rp, ci
    assert 2 * e < 2**31 <= 3 * e
    eps = [(1, 10), (0, 1), (1, 1)]
    tab, cnt = dsg.batch_table([n] * count, [e // 2] * count, [i * (n + 1) for i in range(count)],
                               [i * e for i in range(count)], [i * n for i in range(count)], eps)
    say(f"batch of {count} graphs, {count * e} adjacency entries")
    plan = dsg.Batch(tab, cnt, rp_all.numel(), ci_all.numel(), count * n)
    best = torch.full((count * n,), -7, dtype=torch.int32, device="cuda")
    rem = torch.full((count * n,), -7, dtype=torch.int32, device="cuda")
    res = plan.run(rp_all, ci_all, best_ids=best, removed_at=rem)
    torch.cuda.synchronize()
    got = dsg.Batch.results(res)
    ids = torch.arange(n_side, dtype=torch.int32, device="cuda")
    for i in range(count):
        passes, best_pass, num, den, rem_big, rem_small = expected(n_side, eps[i])
        r = got[i]
        assert r["status"] == 0, (i, r)
        assert (r["passes"], r["best_pass"], r["num"], r["den"]) == (passes, best_pass, num, den), (i, r)
        o = i * n
        assert bool((rem[o:o + n_side] == rem_big).all()) and bool((rem[o + n_side:o + n] == rem_small).all())
        if best_pass == 1:
            assert r["best_size"] == n_side and bool((best[o:o + n_side] == ids).all())
        else:
            assert r["best_size"] == n
    del rp_all, ci_all, best, rem, plan, res
    torch.cuda.empty_cache()


def cbds_expected(n_side: int):
    """CBDS-P of the bridged cliques: core number 32 for the 32-clique part
    (31 clique mates and a bridge), 63 for the 64-clique part; the cores of
    order 33..63 are the 64-clique part (density 63/2 > 24), so K = 33; the
    32-clique vertices are eligible (32 > 31.5) but have one neighbour in the
    core, so none is legitimate."""
    return dict(num=63 * n_side // 2, den=n_side, core_num=63 * n_side // 2, core_den=n_side,
                K=33, kmax=63, n_eligible=n_side, n_legit=0)


def check_cbds(r, n_side):
    import torch
    want = cbds_expected(n_side)
    got = {k: getattr(r, k) for k in want}
    assert got == want, (got, want)
    ids = torch.arange(n_side, dtype=torch.int32, device=r.best.device)
    assert r.best.numel() == n_side and bool((r.best == ids).all())
    assert bool((r.core[:n_side] == 63).all()) and bool((r.core[n_side:] == 32).all())


def test_cbds_closed_form_small_and_just_below_int32_limit():
    import torch
    from paper_2103_00154_amd import dsg
    n_side = 64 * 40
    rp, ci = bridged_cliques(n_side, "cpu")
    g = inputs.Graph(2 * n_side, ci.numel() // 2, rp.numpy(), ci.numpy(), name="bridged")
    o = oracle.cbds(g)
    want = cbds_expected(n_side)
    assert {k: getattr(o, k) for k in want} == want
    check_cbds(dsg.cbds(rp.cuda(), ci.cuda(), core=True), n_side)
    say(f"CBDS-P on bridged cliques with 2m = {96 * N_MAX}")
    rp, ci = bridged_cliques(N_MAX, "cuda")
    check_cbds(dsg.cbds(rp, ci, core=True), N_MAX)
    del rp, ci
    torch.cuda.empty_cache()


def test_star_with_a_hundred_million_leaves():
    # ε = 1/10: threshold floor(2.2 * m / n) = 2, so every leaf fails in
    # pass 1 and its one entry is a degree record for the hub (100 M records
    # for a single survivor rank); the hub, left with degree 0, fails in
    # pass 2; the whole graph (pass 0) stays the best.  CBDS-P: every core
    # number is 1, C_0 = C_1 = G, so K = 0 and the result is G.
    import torch
    from paper_2103_00154_amd import dsg
    leaves = 100_000_000
    n = leaves + 1
    rp = torch.cat([torch.zeros(1, dtype=torch.int64, device="cuda"),
                    leaves + torch.arange(0, n, dtype=torch.int64, device="cuda")]).to(torch.int32)
    ci = torch.cat([torch.arange(1, n, dtype=torch.int32, device="cuda"),
                    torch.zeros(leaves, dtype=torch.int32, device="cuda")])
    say(f"star with {leaves} leaves")
    r = dsg.peel(rp, ci, (1, 10), removed_at=True, trace=True)
    assert (r.passes, r.best_pass, r.num, r.den) == (2, 0, leaves, n)
    assert r.best.numel() == n and bool((r.best == torch.arange(n, dtype=torch.int32, device="cuda")).all())
    assert int(r.removed_at[0]) == 2 and bool((r.removed_at[1:] == 1).all())
    t = r.trace[0]
    assert (t["removed"], t["cross"], t["intra"], t["s_out"], t["e_out"]) == (leaves, leaves, 0, 1, 0)
    c = dsg.cbds(rp, ci, core=True)
    assert (c.num, c.den, c.K, c.kmax, c.n_legit) == (leaves, n, 0, 1, 0)
    assert bool((c.core == 1).all()) and c.best.numel() == n
    del rp, ci, r, c
    torch.cuda.empty_cache()
