"""Helpers shared by the GPU tests: move a generated graph to the device,
run the library and the oracle on it, and compare every output."""
from __future__ import annotations

import sys

import numpy as np

import oracle

INT32_MAX = 2**31 - 1

COMPARED = ("s_in", "e_in", "removed", "cross", "intra", "s_out", "e_out")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_device(g):
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to("cuda")
    ci = torch.from_numpy(np.ascontiguousarray(g.col_idx if g.col_idx.size else
                                                np.zeros(0, np.int32))).to("cuda")
    return rp, ci


def assert_same(r, o, n):
    """GPU result r (PeelResult with removed_at and trace) equals oracle o."""
    assert (r.passes, r.best_pass, r.num, r.den) == (o.passes, o.best_pass, o.num, o.den), (
        (r.passes, r.best_pass, r.num, r.den), (o.passes, o.best_pass, o.num, o.den))
    if r.best is not None:
        assert np.array_equal(r.best.cpu().numpy(), o.best)
    if r.removed_at is not None:
        got = r.removed_at.cpu().numpy()
        assert np.array_equal(got, o.removed_at[:n]), int(np.count_nonzero(got != o.removed_at))
    if r.trace:
        assert len(r.trace) == min(len(o.trace), 4096)
        for k, (a, b) in enumerate(zip(r.trace, o.trace)):
            for f in COMPARED:
                assert a[f] == b[f], (k + 1, f, a[f], b[f])
            assert a["thresh"] == min(b["thresh"], INT32_MAX), (k + 1, a["thresh"], b["thresh"])
            # rows of vertices that fail with degree 0 are not walked, and no
            # row is walked in a pass that leaves no survivor
            if a["s_out"] > 0:
                assert a["cross"] + a["intra"] <= a["walked"] <= b["scanned"]
            else:
                assert a["walked"] == 0


def check(g, eps, **kw):
    from paper_2103_00154_amd import dsg
    say(f"case {g.name} n={g.n} m={g.m} eps={eps[0]}/{eps[1]} {kw}")
    rp, ci = to_device(g)
    r = dsg.peel(rp, ci, eps, removed_at=True, trace=True, **kw)
    o = oracle.peel_graph(g, *eps)
    assert_same(r, o, g.n)
    return r, o
