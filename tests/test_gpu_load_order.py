"""The binding loads the HIP library after torch's HIP runtime, whatever the
caller touches first: a fresh process that asks the library for a workspace
size before any torch device work still peels correctly (loaded the other
way round, the library's HIP runtime would find no device)."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

import pytest

pytestmark = pytest.mark.gpu

ROOT = Path(__file__).resolve().parents[1]

SCRIPT = r"""
import sys
sys.path.insert(0, sys.argv[1])
from paper_2103_00154_amd import dsg, inputs
assert dsg.workspace_bytes(1000, 5000) > 0          # the library is loaded here
import torch, oracle, numpy as np
g = inputs.erdos_renyi(3000, 15000, 7)
rp = torch.from_numpy(g.row_ptr).cuda(); ci = torch.from_numpy(g.col_idx).cuda()
r = dsg.peel(rp, ci, (1, 10))
ws = dsg.alloc_workspace(g.n, g.m)
a = dsg.async_result(dsg.peel_async(rp, ci, (1, 10), workspace=ws)); torch.cuda.synchronize()
o = oracle.peel_graph(g, 1, 10, trace=False)
assert (r.passes, r.num, r.den) == (o.passes, o.num, o.den), (r, o.passes)
assert (a["status"], a["passes"], a["num"], a["den"]) == (0, o.passes, o.num, o.den), a
assert np.array_equal(r.best.cpu().numpy(), o.best)
print("load order ok", flush=True)
"""


def test_library_loaded_before_torch_device_work():
    proc = subprocess.run([sys.executable, "-c", SCRIPT, str(ROOT)], capture_output=True,
                          text=True, timeout=240, env=dict(os.environ))
    print(proc.stdout[-2000:], proc.stderr[-2000:], flush=True)
    assert proc.returncode == 0 and "load order ok" in proc.stdout
