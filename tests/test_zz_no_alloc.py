"""dsg_peel_async_noalloc (the entry point for callers that cannot allocate)
against dsg_peel_async with a caller workspace: the same device result, S~
and removal passes, bit for bit, on two calls in a row (the second on a
smaller graph, over the contents the first left in the static workspace);
also against the oracle, and a graph whose workspace exceeds the static
array is refused with DSG_EINVAL.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
from paper_2103_00154_amd import dsg, inputs

pytestmark = pytest.mark.gpu

LIMIT = 256 << 20  # bytes of the static workspace


def _noalloc(rp, ci, n, m, eps, best, rem, res, head=0):
    import torch
    h = dsg.lib()
    fn = h.dsg_peel_async_noalloc
    fn.argtypes = [ctypes.POINTER(dsg.CSR), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                   ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_void_p]
    fn.restype = ctypes.c_int32
    csr = dsg.CSR(rp.data_ptr(), ci.data_ptr())
    ln = dsg.Launch(0, 0, head, 0) if head else None
    return fn(ctypes.byref(csr), n, m, eps[0], eps[1], best.data_ptr(), rem.data_ptr(),
              res.data_ptr(), ctypes.byref(ln) if ln is not None else None,
              torch.cuda.current_stream().cuda_stream)


def _both(g, eps, head=0):
    import torch
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    outs = []
    for kind in ("noalloc", "workspace"):
        best = torch.full((g.n,), -3, dtype=torch.int32, device="cuda")
        rem = torch.full((g.n,), -3, dtype=torch.int32, device="cuda")
        res = torch.zeros(dsg.RESULT_WORDS, dtype=torch.int64, device="cuda")
        if kind == "noalloc":
            assert _noalloc(rp, ci, g.n, g.m, eps, best, rem, res, head) == dsg.DSG_OK
        else:
            ws = dsg.alloc_workspace(g.n, g.m)
            dsg.peel_async(rp, ci, eps, workspace=ws, best_ids=best, removed_at=rem, result=res,
                           head_passes=head)
        torch.cuda.synchronize()
        outs.append((res.cpu().numpy(), best.cpu().numpy(), rem.cpu().numpy()))
    (ra, ba, ma), (rb, bb, mb) = outs
    assert np.array_equal(ra, rb)
    assert np.array_equal(ba, bb) and np.array_equal(ma, mb)
    r = dsg.async_result(torch.from_numpy(ra))
    o = oracle.peel_graph(g, *eps, trace=False)
    assert (r["status"], r["passes"], r["best_pass"], r["num"], r["den"]) == (
        0, o.passes, o.best_pass, o.num, o.den)
    assert np.array_equal(ba[:r["best_size"]], o.best)
    assert np.array_equal(ma, o.removed_at)
    print(f"noalloc {g.name} eps={eps[0]}/{eps[1]} head={head}: passes {r['passes']} "
          f"best {r['num']}/{r['den']} == workspace call == oracle", flush=True)


def test_two_calls_in_a_row_the_second_smaller():
    big = inputs.rmat(20, 16, seed=0)
    assert dsg.workspace_bytes(big.n, big.m) <= LIMIT
    _both(big, (1, 10))
    _both(inputs.erdos_renyi(10_000, 50_000, 0), (1, 10))
    _both(inputs.chung_lu(3000, 12, 2.3, 4), (0, 1), head=1)


def test_graph_too_large_for_the_static_workspace():
    import torch
    n, m = 1 << 22, 1 << 25
    assert dsg.workspace_bytes(n, m) > LIMIT
    rp = torch.zeros(8, dtype=torch.int32, device="cuda")
    t = torch.zeros(8, dtype=torch.int32, device="cuda")
    res = torch.zeros(dsg.RESULT_WORDS, dtype=torch.int64, device="cuda")
    assert _noalloc(rp, t, n, m, (1, 10), t, t, res) == dsg.DSG_EINVAL
