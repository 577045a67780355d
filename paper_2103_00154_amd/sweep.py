"""eps sweeps of the peel (Section 4.3 runs P-Bahmani at several eps values,
eps = 0 included): one device graph, a list of eps = num/den values, and for
each the result, the per-pass trace and the device time.

A smaller eps lowers the removal threshold 2(1+eps)rho, so fewer vertices fail
per pass: more passes, and a kept graph at least as close to the densest one
in practice (the guarantee rho(S~) >= rho* / (2 + 2 eps) tightens).  With
eps = 0 the pass count is bounded by n instead of log_{1+eps} n.

With ``exact=True`` the sweep also computes rho* on the device
(dsg_exact_density, Goldberg's construction of Section 2) and reports
rho(S~) / rho* for every eps, the accuracy Section 4 compares.
"""
from __future__ import annotations

import statistics
from dataclasses import dataclass, field

from . import dsg

DEFAULT_EPS = ((0, 1), (1, 100), (1, 20), (1, 10), (1, 2), (1, 1), (2, 1))


@dataclass
class SweepPoint:
    eps: tuple
    passes: int
    best_pass: int
    num: int
    den: int
    ms: float
    trace: list = field(default_factory=list)
    ratio: float | None = None  # rho(S~) / rho*, when rho* was computed

    @property
    def density(self) -> float:
        return self.num / self.den if self.den else 0.0


def eps_sweep(row_ptr, col_idx, eps_list=DEFAULT_EPS, *, reps: int = 3, workspace=None,
              best_ids=None, exact: bool = False) -> list[SweepPoint]:
    """Peel the device graph once per eps with the trace, then `reps` more
    times for the median device time (HIP events on the current stream);
    with ``exact`` also rho(S~) / rho* from the device's exact rho*."""
    import torch
    n = row_ptr.numel() - 1
    m = col_idx.numel() // 2
    if workspace is None:
        workspace = dsg.alloc_workspace(n, m, row_ptr.device)
    if best_ids is None:
        best_ids = torch.empty(max(n, 1), dtype=torch.int32, device=row_ptr.device)
    out = []
    for eps in eps_list:
        r = dsg.peel(row_ptr, col_idx, eps, best_ids=best_ids, workspace=workspace, trace=True)
        times = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            z = torch.cuda.Event(enable_timing=True)
            a.record()
            dsg.peel(row_ptr, col_idx, eps, best_ids=best_ids, workspace=workspace)
            z.record()
            z.synchronize()
            times.append(a.elapsed_time(z))
        out.append(SweepPoint(tuple(eps), r.passes, r.best_pass, r.num, r.den,
                              statistics.median(times) if times else 0.0, r.trace))
    if exact:
        x = dsg.exact_density(row_ptr, col_idx, extract=False)
        for pt in out:
            pt.ratio = (pt.num * x.den) / (pt.den * x.num) if pt.den and x.num else 1.0
    return out
