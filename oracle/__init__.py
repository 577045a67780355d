"""CPU oracle for Bahmani's (2+2eps) peeling (Algorithm 1, P-Bahmani).

TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library and never imports it.

* :func:`peel`            - the sequential C oracle (``peel_oracle.c``).
* :mod:`oracle.literal`   - the same method recomputing every degree and
                            edge count from its definition in each pass
                            (pure Python, tiny graphs only).
* :mod:`oracle.exact`     - exact densest-subgraph densities (brute force,
                            Goldberg's max-flow construction) used to check
                            the approximation guarantee.
* :func:`cbds`            - CBDS-P (Algorithm 2): densest k-core extended by
                            legitimate vertices (``cbds_oracle.c``).
* :mod:`oracle.cbds_literal` - the same from the definitions of the k-core and
                            of the extension step (pure Python, small graphs).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_P = ctypes.c_void_p

NEVER = 2**31 - 1

TRACE_FIELDS = ("s_in", "e_in", "thresh", "removed", "cross", "intra", "scanned", "s_out", "e_out")


class _Result(ctypes.Structure):
    _fields_ = [("dens_num", _I64), ("dens_den", _I64), ("passes", _I32), ("best_pass", _I32),
                ("best_size", _I64)]


class _Pass(ctypes.Structure):
    _fields_ = [(f, _I64) for f in TRACE_FIELDS]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(str(_build.ensure()))
        lib.dsg_oracle_peel.argtypes = [_P, _P, _I64, _I64, _I64, _P, _P, _P, _I64,
                                        ctypes.POINTER(_Result)]
        lib.dsg_oracle_peel.restype = _I32
        lib.dsg_oracle_check_csr.argtypes = [_P, _P, _I64]
        lib.dsg_oracle_check_csr.restype = _I32
        lib.dsg_oracle_cbds.argtypes = [_P, _P, _I64, _P, _P, _P]
        lib.dsg_oracle_cbds.restype = _I32
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle returned status {code}")
        self.code = code


@dataclass
class OracleResult:
    num: int            # |E(S~)|
    den: int            # |S~|
    passes: int
    best_pass: int
    best: np.ndarray    # S~, ascending int32
    removed_at: np.ndarray  # int32[n], pass in which each vertex failed
    trace: list = field(default_factory=list)  # list of dicts, one per pass


def _arr(x):
    return np.ascontiguousarray(x, dtype=np.int32)


def check_csr(row_ptr, col_idx, n: int) -> int:
    rp, ci = _arr(row_ptr), _arr(col_idx)
    return int(_load().dsg_oracle_check_csr(rp.ctypes.data, ci.ctypes.data if ci.size else None, n))


def peel(row_ptr, col_idx, n: int, eps_num: int, eps_den: int, trace: bool = True) -> OracleResult:
    """Run the C oracle on host arrays.  ``eps = eps_num / eps_den``."""
    lib = _load()
    rp, ci = _arr(row_ptr), _arr(col_idx)
    removed = np.empty(max(n, 1), dtype=np.int32)
    best = np.empty(max(n, 1), dtype=np.int32)
    cap = n + 1 if trace else 0
    tr = (_Pass * max(cap, 1))()
    res = _Result()
    rc = lib.dsg_oracle_peel(rp.ctypes.data if rp.size else None,
                             ci.ctypes.data if ci.size else None, n, eps_num, eps_den,
                             removed.ctypes.data, best.ctypes.data,
                             ctypes.addressof(tr) if trace else None, cap, ctypes.byref(res))
    if rc != 0:
        raise OracleError(rc)
    passes = []
    if trace:
        for k in range(res.passes):
            passes.append({f: int(getattr(tr[k], f)) for f in TRACE_FIELDS})
    return OracleResult(num=res.dens_num, den=res.dens_den, passes=res.passes,
                        best_pass=res.best_pass, best=best[:res.best_size].copy(),
                        removed_at=removed[:n].copy(), trace=passes)


def peel_graph(g, eps_num: int, eps_den: int, trace: bool = True) -> OracleResult:
    return peel(g.row_ptr, g.col_idx, g.n, eps_num, eps_den, trace=trace)


@dataclass
class CbdsResult:
    num: int            # |E(S)| of the result S = C_K u L
    den: int            # |S|
    core_num: int       # |E(C_K)|
    core_den: int       # |C_K|
    K: int              # order of the densest core
    n_legit: int        # |L|
    kmax: int           # largest core number
    best: np.ndarray    # S, ascending int32
    core: np.ndarray    # core number of every vertex
    n_eligible: int
    legit_edges: int    # sum of legits over L plus |E(L)|


def cbds(g) -> CbdsResult:
    """CBDS-P (Section 3.2, Algorithm 2) of a Graph from ``inputs``."""
    lib = _load()
    n = g.n
    core = np.empty(max(n, 1), dtype=np.int32)
    best = np.empty(max(n, 1), dtype=np.int32)
    out = np.zeros(10, dtype=np.int64)
    rp = _arr(g.row_ptr)
    ci = _arr(g.col_idx if g.col_idx.size else np.zeros(1, np.int32))
    rc = lib.dsg_oracle_cbds(rp.ctypes.data, ci.ctypes.data, n, core.ctypes.data,
                             best.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    o = [int(x) for x in out]
    return CbdsResult(num=o[0], den=o[1], core_num=o[2], core_den=o[3], K=o[4], n_legit=o[5],
                      kmax=o[6], best=best[:o[7]].copy(), core=core[:n].copy(), n_eligible=o[8],
                      legit_edges=o[9])
