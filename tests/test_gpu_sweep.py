"""eps sweeps on the GPU (Section 4.3 runs the peel at several eps, eps = 0
included): every point of a sweep equals the oracle, per-pass trace
included, and on graphs small enough for the exact densest subgraph
(Goldberg's construction in the oracle) every point meets its (2 + 2 eps)
guarantee; the measured approximation ratios are printed.
"""
from __future__ import annotations

import pytest

import oracle
from gpu_util import COMPARED, INT32_MAX, say, to_device
from oracle import exact
from paper_2103_00154_amd import inputs

pytestmark = pytest.mark.gpu

EPS = ((0, 1), (1, 100), (1, 20), (1, 10), (1, 2), (1, 1), (2, 1), (5, 1))


def test_sweep_matches_oracle_pass_by_pass():
    from paper_2103_00154_amd import sweep
    g = inputs.rmat(18, 16, seed=5)
    rp, ci = to_device(g)
    pts = sweep.eps_sweep(rp, ci, EPS, reps=1)
    for pt in pts:
        o = oracle.peel_graph(g, *pt.eps)
        assert (pt.passes, pt.best_pass, pt.num, pt.den) == (o.passes, o.best_pass, o.num, o.den)
        assert len(pt.trace) == len(o.trace)
        for a, b in zip(pt.trace, o.trace):
            for f in COMPARED:
                assert a[f] == b[f], (pt.eps, f)
            assert a["thresh"] == min(b["thresh"], INT32_MAX)
        say(f"eps {pt.eps[0]}/{pt.eps[1]}: passes {pt.passes}, best {pt.num}/{pt.den} "
            f"(pass {pt.best_pass}), {pt.ms:.3f} ms")


@pytest.mark.parametrize("gi", range(4))
def test_sweep_meets_the_guarantee_against_the_exact_densest(gi):
    from paper_2103_00154_amd import sweep
    g = [inputs.chung_lu(1500, 12, 2.2, seed=3),
         inputs.erdos_renyi(1200, 9000, 4),
         inputs.rmat(11, 8, seed=6),
         inputs.rmat(11, 16, seed=7, planted=(40, 0.6, 8))][gi]
    e_star, s_star, _ = exact.densest_goldberg(g.n, g.edges())
    rp, ci = to_device(g)
    for pt in sweep.eps_sweep(rp, ci, EPS, reps=1, exact=True):
        num, den = pt.eps
        # the ratio the sweep reports from the GPU's rho* is the oracle's
        assert abs(pt.ratio - pt.num * s_star / (pt.den * e_star)) < 1e-12
        # rho(S~) >= rho* / (2 + 2 eps), in integers
        assert 2 * (num + den) * pt.num * s_star >= den * e_star * pt.den, pt.eps
        say(f"{g.name} eps {num}/{den}: rho(S~) / rho* = "
            f"{pt.num * s_star / (pt.den * e_star):.4f} (bound {den / (2 * (num + den)):.4f})")
