"""Full-size parity: R-MAT scale 24 (n = 16,777,216, edge factor 16,
(a,b,c,d) = (.57,.19,.19,.05), seed 0) with a planted G(2000, 1/2) block on
random ids (seed 1), eps = 1/10, run exactly as the benchmark runs it
(default launch shape, caller workspace, extraction on).  The oracle
finishes this graph in seconds, so every output is compared, not a sample.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import assert_same, say, to_device
from paper_2103_00154_amd import inputs

pytestmark = pytest.mark.gpu


def test_rmat24_planted_full_parity():
    import torch
    from paper_2103_00154_amd import dsg
    say("case rmat24+planted2000 eps=1/10: generating")
    g = inputs.rmat(24, 16, seed=0, planted=(2000, 0.5, 1))
    say(f"n={g.n} m={g.m}; oracle")
    o = oracle.peel_graph(g, 1, 10)
    say(f"oracle passes={o.passes} best={o.num}/{o.den}; GPU")
    rp, ci = to_device(g)
    ws = dsg.alloc_workspace(g.n, g.m)
    best = torch.empty(g.n, dtype=torch.int32, device="cuda")
    rem = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for rep in range(2):
        r = dsg.peel(rp, ci, (1, 10), best_ids=best, removed_at=rem, trace=True, workspace=ws)
        assert_same(r, o, g.n)
        say(f"rep {rep} ok")
    # the planted block's density is within the (2+2eps) factor of S~
    ids = g.meta["planted_ids"]
    e = g.edges()
    mask = np.zeros(g.n, dtype=bool)
    mask[ids] = True
    e_p = int(np.count_nonzero(mask[e[:, 0]] & mask[e[:, 1]]))
    assert 2 * 11 * r.num * len(ids) >= 10 * e_p * r.den
    overlap = int(np.count_nonzero(mask[r.best.cpu().numpy()]))
    say(f"planted density {e_p}/{len(ids)}; S~ {r.num}/{r.den}; |S~ & P| = {overlap}")


@pytest.mark.parametrize("eps", [(1, 10), (0, 1)])
def test_power_law_graph_with_id_keyed_passes_by_default(eps):
    # a Chung-Lu graph of 5 M vertices: its first pass leaves more than
    # 65,536 survivors and walks more than 2^25 entries, so by default it
    # keys its degree records by neighbour id, and later passes gather
    # survivor ranks; every output is compared with the oracle
    from paper_2103_00154_amd import dsg
    g = inputs.chung_lu(5_000_000, 24, 2.3, 5)
    say(f"case chung_lu n={g.n} m={g.m} eps={eps[0]}/{eps[1]}: oracle")
    o = oracle.peel_graph(g, *eps)
    rp, ci = to_device(g)
    r = dsg.peel(rp, ci, eps, removed_at=True, trace=True)
    assert any(t["s_out"] > 65536 and t["walked"] >= 1 << 25 for t in r.trace), r.trace[:2]
    assert_same(r, o, g.n)
