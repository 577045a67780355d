"""Serving on the GPU: requests arriving as a Poisson stream are admitted by
HBM footprint, batched as they come on several streams, and every result is
bit-identical to peeling the same graph alone (the single-graph path), and
to the oracle on a sample.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import say
from paper_2103_00154_amd import inputs

pytestmark = pytest.mark.gpu

EPS = ((1, 100), (1, 10), (1, 2))


def _pool(count, seed, median, cap):
    specs = inputs.serving_specs(count, seed=seed, median=median, n_cap=cap)
    b = inputs.make_batch(specs)
    return [b.graph(i) for i in range(b.count)]


def _alone(graphs):
    """(graph index, eps) -> result of the single-graph path."""
    import torch
    from paper_2103_00154_amd import dsg
    out = {}
    for gi, g in enumerate(graphs):
        rp = torch.from_numpy(g.row_ptr).cuda()
        ci = torch.from_numpy(g.col_idx if g.m else np.zeros(1, np.int32)).cuda()
        for e in EPS:
            r = dsg.peel(rp, ci, e, m=g.m)
            out[(gi, e)] = (r.num, r.den, r.passes, r.best_pass, r.best.cpu().numpy())
    return out


def _check(reqs, graphs, alone):
    for rq in reqs:
        gi = rq.rid % len(graphs)
        num, den, passes, bp, best = alone[(gi, rq.eps)]
        r = rq.result
        assert r["status"] == 0, (rq.rid, r)
        assert (r["num"], r["den"], r["passes"], r["best_pass"]) == (num, den, passes, bp), rq.rid
        assert np.array_equal(rq.best, best), rq.rid


def test_continuous_batching_matches_alone_results():
    import torch
    from paper_2103_00154_amd import serve
    graphs = _pool(48, seed=1, median=3000, cap=120_000)
    say(f"pool: {len(graphs)} graphs, n max {max(g.n for g in graphs)}, "
        f"m total {sum(g.m for g in graphs)}")
    alone = _alone(graphs)
    hg = [serve.HostGraph.from_graph(g) for g in graphs]
    # a budget of a few graphs' footprint: admission must hold requests back
    budget = 6 * max(serve.footprint(g.n, g.m) for g in graphs)
    srv = serve.Server(budget, streams=4, max_batch=32)
    reqs = serve.run_load(srv, hg, EPS, qps=20_000, count=300, seed=2)
    srv.close()
    torch.cuda.synchronize()
    st = serve.latency_stats(reqs)
    say(f"stats {st}; batches {srv.batches}, max batch {max(srv.batch_sizes)}, "
        f"max in flight {srv.max_in_flight}, arena peak {srv.arena.peak} of {srv.arena.size}")
    assert len(srv.completed) == 300 and all(r.done > 0 for r in reqs)
    assert srv.max_in_flight >= 2          # batches overlapped on the device
    assert max(srv.batch_sizes) > 1        # requests were batched
    assert srv.arena.peak <= srv.arena.size and srv.arena.used == 0
    _check(reqs, graphs, alone)
    # the oracle agrees on a sample
    for rq in reqs[:12]:
        g = graphs[rq.rid % len(graphs)]
        o = oracle.peel_graph(g, *rq.eps, trace=False)
        assert (rq.result["num"], rq.result["den"], rq.result["passes"]) == (o.num, o.den, o.passes)
        assert np.array_equal(rq.best, o.best)


def test_same_results_alone_and_in_a_mix_of_sizes():
    import torch
    from paper_2103_00154_amd import serve
    # small graphs mixed with graphs larger than the LDS vertex state
    graphs = _pool(10, seed=4, median=1500, cap=50_000)
    graphs += [inputs.chung_lu(150_000, 24, 2.3, seed=77), inputs.erdos_renyi(90_000, 500_000, 78)]
    alone = _alone(graphs)
    hg = [serve.HostGraph.from_graph(g) for g in graphs]
    for lane in (True, False):
        # with the single-graph lane for the large graphs, and without it
        srv = serve.Server(1 << 30, streams=3, max_batch=8,
                           big_vertices=None if lane else 0)
        reqs = serve.run_load(srv, hg, EPS, qps=5_000, count=96, seed=5)
        srv.close()
        torch.cuda.synchronize()
        say(f"lane {lane}: stats {serve.latency_stats(reqs)}; batches {srv.batches}, "
            f"large-graph lane {srv.big_done}")
        assert (srv.big_done > 0) == lane
        assert srv.arena.used == 0
        _check(reqs, graphs, alone)


def test_request_larger_than_the_budget_is_refused():
    from paper_2103_00154_amd import serve
    g = inputs.erdos_renyi(2000, 10_000, 1)
    srv = serve.Server(64 * 1024, streams=1)
    with pytest.raises(ValueError):
        srv.submit(serve.Request(0, serve.HostGraph.from_graph(g), (1, 10), 0.0))


def test_large_requests_overflow_into_batches_when_the_lane_is_backed_up():
    import torch
    from paper_2103_00154_amd import serve
    # only graphs larger than the LDS vertex state, all arriving at once, one
    # lane stream and overflow on: the lane's queue backs up and later
    # requests overflow into micro-batches of their own on the batch kernel
    graphs = [inputs.chung_lu(150_000, 16, 2.3, seed=81), inputs.erdos_renyi(100_000, 300_000, 82),
              inputs.chung_lu(120_000, 24, 2.6, seed=83)]
    alone = _alone(graphs)
    hg = [serve.HostGraph.from_graph(g) for g in graphs]
    srv = serve.Server(4 << 30, streams=4, max_batch=8, big_lanes=1, overflow=True)
    assert all(g.n > srv.big_vertices for g in graphs)
    reqs = serve.run_load(srv, hg, EPS, qps=1e6, count=24, seed=6)
    srv.close()
    torch.cuda.synchronize()
    say(f"stats {serve.latency_stats(reqs)}; lane {srv.big_done}, overflowed {srv.overflowed}")
    assert srv.overflowed > 0 and srv.big_done > 0
    assert srv.overflowed + srv.big_done == 24
    assert srv.arena.used == 0
    _check(reqs, graphs, alone)


def test_load_beyond_capacity_is_shed_and_served_results_stay_exact():
    import torch
    from paper_2103_00154_amd import serve
    # far more requests per second than the device serves: requests that
    # wait more than 20 ms are rejected; the rest keep a bounded latency and
    # their results are exact
    graphs = _pool(32, seed=9, median=20_000, cap=400_000)
    alone = _alone(graphs)
    hg = [serve.HostGraph.from_graph(g) for g in graphs]
    srv = serve.Server(8 << 30, streams=4, max_batch=64, max_queue_s=0.02)
    reqs = serve.run_load(srv, hg, EPS, qps=200_000, count=2000, seed=10)
    torch.cuda.synchronize()
    st = serve.latency_stats(reqs)
    say(f"stats {st}; lane {srv.big_done}, rejected {srv.rejected}")
    assert st["rejected"] > 0 and st["served"] > 0
    assert st["served"] + st["rejected"] == 2000 and srv.arena.used == 0
    served = [r for r in reqs if not r.rejected]
    # admitted within the shedding bound (checked at every tick)
    assert max(r.admitted - r.arrival for r in served) < 0.02 + 0.05
    _check(served, graphs, alone)
