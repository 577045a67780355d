"""The launch-shape autotuner: it times every candidate on the batch, picks
a supported shape, stores and reuses the winner per device and batch
signature, and the chosen shape gives the oracle's results."""
from __future__ import annotations

import json

import numpy as np
import pytest

import oracle
from paper_2103_00154_amd import inputs

pytestmark = pytest.mark.gpu


def test_autotune_picks_a_supported_shape_and_caches_it(tmp_path):
    import torch
    from paper_2103_00154_amd import autotune, dsg
    b = inputs.make_batch(inputs.batch_specs(40, seed=11, n_range=(100, 8000)))
    rp = torch.from_numpy(b.row_ptr).cuda()
    ci = torch.from_numpy(b.col_idx).cuda()
    tab, count = dsg.batch_table(b.n, b.m, b.rp_off, b.ci_off, b.out_off, (1, 10))
    sig = autotune.batch_signature(b.n, b.m)
    cache = tmp_path / "tune.json"
    cands = autotune.CANDIDATES[:6]
    win, timings = autotune.tune_batch(tab, count, len(b.row_ptr), len(b.col_idx), b.out_len,
                                       rp, ci, candidates=cands, reps=2, cache=cache,
                                       signature=sig)
    assert len(timings) == len(cands) and all(ms > 0 for ms, _ in timings)
    assert win in [{k: c[k] for k in ("block", "walk_items", "blocks_per_cu")} for c in cands]
    assert json.loads(cache.read_text())  # stored
    again, t2 = autotune.tune_batch(tab, count, len(b.row_ptr), len(b.col_idx), b.out_len, rp,
                                    ci, candidates=cands, cache=cache, signature=sig)
    assert again == win and t2 == []      # reused without timing
    plan = dsg.Batch(tab, count, len(b.row_ptr), len(b.col_idx), b.out_len, launch=win)
    best = torch.empty(b.out_len, dtype=torch.int32, device="cuda")
    res = dsg.Batch.results(plan.run(rp, ci, best_ids=best))
    h = best.cpu().numpy()
    for i in range(count):
        o = oracle.peel_graph(b.graph(i), 1, 10, trace=False)
        a = int(b.out_off[i])
        assert (res[i]["num"], res[i]["den"], res[i]["passes"]) == (o.num, o.den, o.passes)
        assert np.array_equal(h[a:a + res[i]["best_size"]], o.best)
