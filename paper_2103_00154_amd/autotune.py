"""Launch-shape autotuner for the batched peel (dsg_batch_prepare).

The persistent batch kernel has three shape parameters that trade LDS for
parallelism: threads per workgroup, adjacency entries per lane per wave
tile, and workgroups resident per CU (which splits the CU's LDS, and so the
number of vertices whose state fits in LDS).  The best choice depends on the
batch's size mix, so it is measured: every candidate shape runs the actual
batch a few times on the device and the fastest median wins.  Results never
depend on the shape (the kernels are exact), only the time does.

Tuning outcomes can be kept in a JSON file keyed by device name and a coarse
signature of the batch, so that a serving process tunes a batch class once.
"""
from __future__ import annotations

import json
import math
import statistics
from pathlib import Path

from . import dsg

#: candidate shapes, every (block, walk_items, blocks_per_cu) the library supports
CANDIDATES = tuple(
    {"block": blk, "walk_items": it, "blocks_per_cu": bpc}
    for blk in (256, 512, 1024)
    for it in (4, 8, 16)
    for bpc in (1, 2, 4)
    if not (blk == 1024 and it == 16) and blk * bpc <= 2048
)


def batch_signature(n, m) -> str:
    """Coarse class of a batch: graph count and log2 buckets of its total and
    largest vertex and edge counts."""
    import numpy as np
    n = np.asarray(n, dtype=np.int64)
    m = np.asarray(m, dtype=np.int64)
    def b(x):
        return int(math.log2(max(int(x), 1)))
    return (f"c{b(len(n))}-n{b(n.sum())}-m{b(m.sum())}-nmax{b(n.max() if len(n) else 0)}"
            f"-mmax{b(m.max() if len(m) else 0)}")


def _time_shape(table, count, rp_len, ci_len, out_len, rp, ci, best, res, launch, reps,
                workspace):
    import torch
    plan = dsg.Batch(table, count, rp_len, ci_len, out_len, launch=launch, workspace=workspace)
    plan.run(rp, ci, best_ids=best, results=res)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record()
        plan.run(rp, ci, best_ids=best, results=res)
        z.record()
        z.synchronize()
        times.append(a.elapsed_time(z))
    return statistics.median(times), plan.shape


def tune_batch(table, count: int, rp_len: int, ci_len: int, out_len: int, rp, ci, *,
               candidates=CANDIDATES, reps: int = 3, cache: str | Path | None = None,
               signature: str | None = None, log=None) -> tuple[dict, list]:
    """Time every candidate shape on this batch; return (best launch dict,
    [(ms, shape), ...] for all candidates).  With ``cache`` (a JSON path) and
    ``signature``, a stored winner for this device and signature is returned
    without timing, and a new winner is stored."""
    import torch
    key = None
    if cache is not None and signature is not None:
        key = f"{torch.cuda.get_device_name()}|{signature}"
        p = Path(cache)
        if p.exists():
            try:
                stored = json.loads(p.read_text()).get(key)
            except ValueError:
                stored = None
            if stored:
                return dict(stored), []
    best = torch.empty(max(out_len, 1), dtype=torch.int32, device=rp.device)
    res = torch.empty((max(count, 1), dsg.RESULT_WORDS), dtype=torch.int64, device=rp.device)
    entries = sum(2 * int(table[i].m) for i in range(count))
    workspace = torch.empty(dsg.batch_workspace_bytes(count, entries, out_len), dtype=torch.uint8,
                            device=rp.device)
    timings = []
    for launch in candidates:
        ms, shape = _time_shape(table, count, rp_len, ci_len, out_len, rp, ci, best, res,
                                launch, reps, workspace)
        timings.append((ms, shape))
        if log:
            log(f"  shape {launch}: {ms:.3f} ms (LDS vertices {shape['lds_vertices']})")
    ms, shape = min(timings, key=lambda t: t[0])
    win = {k: shape[k] for k in ("block", "walk_items", "blocks_per_cu")}
    if key is not None:
        p = Path(cache)
        data = {}
        if p.exists():
            try:
                data = json.loads(p.read_text())
            except ValueError:
                data = {}
        data[key] = win
        p.write_text(json.dumps(data, indent=1, sort_keys=True))
    return win, timings
