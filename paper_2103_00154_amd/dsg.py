"""Python binding of libdsg.so (include/dsg.h): argument marshalling only.

Every step of the peel runs in the library's HIP kernels.  torch supplies
device memory and the current HIP stream.  If the library is missing or fails
to load, every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from pathlib import Path

from . import _build

_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_P = ctypes.c_void_p
_SZ = ctypes.c_size_t

DSG_OK = 0
DSG_EINVAL = -1
DSG_EOVERFLOW = -2
DSG_ENOMEM = -3
DSG_EDEVICE = -4
DSG_EINTERNAL = -5

#: every symbol include/dsg.h declares
EXPORTS = ("dsg_version", "dsg_strerror", "dsg_workspace_bytes", "dsg_peel", "dsg_peel_ex",
           "dsg_validate_csr", "dsg_cbds", "dsg_batch_workspace_bytes", "dsg_batch_prepare",
           "dsg_batch_run", "dsg_peel_async", "dsg_peel_async_noalloc",
           "dsg_exact_workspace_bytes", "dsg_exact_density")

TRACE_FIELDS = ("s_in", "e_in", "thresh", "removed", "cross", "intra", "walked", "s_out", "e_out")


class CSR(ctypes.Structure):
    _fields_ = [("row_ptr", _P), ("col_idx", _P)]


class Result(ctypes.Structure):
    _fields_ = [("dens_num", _I64), ("dens_den", _I64), ("passes", _I32), ("best_pass", _I32),
                ("best_size", _I64)]


class PassTrace(ctypes.Structure):
    _fields_ = [(f, _I64) for f in TRACE_FIELDS]


class Launch(ctypes.Structure):
    _fields_ = [("mark_grid", _I32), ("walk_grid", _I32), ("pass_batch", _I32),
                ("flags", _I32)]


#: dsg_launch.flags bit: keep degree-update records in per-bin regions
LAUNCH_BIN_REGIONS = 1
LAUNCH_NO_PROGRESS = 2
#: dsg_launch.flags bits: degree-update records keyed by neighbour id in
#: every pass that leaves survivors (graphs of at most 2^25 vertices), or never
#: (by default: passes that leave more than 65536 survivors and walk at least
#: 2^25 adjacency entries)
LAUNCH_ID_BUCKETS = 4
LAUNCH_NO_ID_BUCKETS = 8


class Profile(ctypes.Structure):
    _fields_ = [("ms_init", ctypes.c_double), ("ms_mark", ctypes.c_double),
                ("ms_walk", ctypes.c_double), ("ms_apply", ctypes.c_double),
                ("ms_extract", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("launches_walk", _I32), ("launches_mark", _I32), ("launches_apply", _I32),
                ("reserved", _I32), ("walked", _I64), ("cross", _I64),
                ("live_scanned", _I64), ("walk_list", _I64)]


class CbdsResult(ctypes.Structure):
    _fields_ = [("dens_num", _I64), ("dens_den", _I64), ("core_num", _I64), ("core_den", _I64),
                ("core_k", _I32), ("kmax", _I32), ("passes", _I32), ("reserved", _I32),
                ("n_eligible", _I64), ("n_legit", _I64), ("best_size", _I64)]


class BatchGraph(ctypes.Structure):
    _fields_ = [("row_ptr_off", _I64), ("col_idx_off", _I64), ("out_off", _I64), ("n", _I64),
                ("m", _I64), ("eps_num", _I64), ("eps_den", _I64), ("reserved", _I64)]


class BatchResult(ctypes.Structure):
    _fields_ = [("dens_num", _I64), ("dens_den", _I64), ("passes", _I32), ("best_pass", _I32),
                ("best_size", _I64), ("status", _I32), ("reserved", _I32)]


class BatchLaunch(ctypes.Structure):
    _fields_ = [("block", _I32), ("blocks_per_cu", _I32), ("grid", _I32), ("walk_items", _I32)]


class BatchPlan(ctypes.Structure):
    _fields_ = [("count", _I32), ("block", _I32), ("blocks_per_cu", _I32), ("grid", _I32),
                ("walk_items", _I32), ("lds_bytes", _I32), ("lds_vertices", _I32),
                ("state_bits", _I32), ("out_len", _I64), ("workspace", _P),
                ("ws_bytes", ctypes.c_uint64), ("reserved", _I64 * 4)]


class ExactResult(ctypes.Structure):
    _fields_ = [("dens_num", _I64), ("dens_den", _I64), ("set_size", _I64), ("flows", _I32),
                ("relabels", _I32)]


class DsgError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        text = lib().dsg_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {text} (status {status})" if what else text)
        self.status = status


_lib = None


def library_path() -> Path:
    return _build.LIB_DSG


def lib():
    """The loaded ctypes handle of libdsg.so (built first if absent)."""
    global _lib
    if _lib is None:
        path = _build.ensure_dsg()
        # torch brings its own HIP runtime with the same soname as the one
        # the library is linked against (libamdhip64.so.7); whichever is
        # loaded first serves both.  torch goes first, so that the library
        # and torch share one runtime: torch's device pointers and streams
        # belong to it (loaded the other way round, the library's runtime
        # finds no device).
        import torch  # noqa: F401
        try:
            h = ctypes.CDLL(str(path))
        except OSError as exc:  # no silent fallback
            raise RuntimeError(f"cannot load the HIP peeling library {path}: {exc}") from exc
        h.dsg_version.argtypes = []
        h.dsg_version.restype = _I32
        h.dsg_strerror.argtypes = [_I32]
        h.dsg_strerror.restype = ctypes.c_char_p
        h.dsg_workspace_bytes.argtypes = [_I64, _I64]
        h.dsg_workspace_bytes.restype = _SZ
        h.dsg_peel.argtypes = [ctypes.POINTER(CSR), _I64, _I64, _I64, _I64, _P,
                               ctypes.POINTER(Result), _P, _SZ, _P]
        h.dsg_peel.restype = _I32
        h.dsg_peel_ex.argtypes = [ctypes.POINTER(CSR), _I64, _I64, _I64, _I64, _P, _P,
                                  ctypes.POINTER(Result), _P, _I32, _P, _P, _P, _SZ, _P]
        h.dsg_peel_ex.restype = _I32
        h.dsg_validate_csr.argtypes = [ctypes.POINTER(CSR), _I64, _I64, ctypes.POINTER(_I32), _P]
        h.dsg_validate_csr.restype = _I32
        h.dsg_cbds.argtypes = [ctypes.POINTER(CSR), _I64, _I64, _P, _P, ctypes.POINTER(CbdsResult),
                               _P, _I32, _P, _SZ, _P]
        h.dsg_cbds.restype = _I32
        h.dsg_batch_workspace_bytes.argtypes = [_I32, _I64, _I64]
        h.dsg_batch_workspace_bytes.restype = _SZ
        h.dsg_batch_prepare.argtypes = [_P, _I32, _I64, _I64, _I64, _P, _P, _SZ, _P,
                                        ctypes.POINTER(BatchPlan)]
        h.dsg_batch_prepare.restype = _I32
        h.dsg_batch_run.argtypes = [ctypes.POINTER(BatchPlan), _P, _P, _P, _P, _P, _P]
        h.dsg_batch_run.restype = _I32
        h.dsg_peel_async.argtypes = [ctypes.POINTER(CSR), _I64, _I64, _I64, _I64, _P, _P, _P, _P,
                                     _P, _SZ, _P]
        h.dsg_peel_async.restype = _I32
        h.dsg_peel_async_noalloc.argtypes = [ctypes.POINTER(CSR), _I64, _I64, _I64, _I64, _P, _P,
                                             _P, _P, _P]
        h.dsg_peel_async_noalloc.restype = _I32
        h.dsg_exact_workspace_bytes.argtypes = [_I64, _I64]
        h.dsg_exact_workspace_bytes.restype = _SZ
        h.dsg_exact_density.argtypes = [ctypes.POINTER(CSR), _I64, _I64, _P,
                                        ctypes.POINTER(ExactResult), _P, _SZ, _P]
        h.dsg_exact_density.restype = _I32
        _lib = h
    return _lib


def workspace_bytes(n: int, m: int) -> int:
    return int(lib().dsg_workspace_bytes(n, m))


@dataclass
class PeelResult:
    best: object            # torch.int32 device tensor, S~ ascending (None if not extracted)
    num: int                # |E(S~)|
    den: int                # |S~|
    passes: int
    best_pass: int
    removed_at: object = None  # torch.int32 device tensor or None
    trace: list = field(default_factory=list)
    profile: dict | None = None

    @property
    def density(self) -> float:
        return self.num / self.den if self.den else 0.0


def _check_int32_cuda(name, t):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_cuda:
        raise TypeError(f"{name} must be a torch.int32 tensor on a HIP device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def alloc_workspace(n: int, m: int, device=None):
    """A torch uint8 tensor sized for dsg_peel on a graph with (n, m)."""
    import torch
    nbytes = workspace_bytes(n, m)
    if nbytes == 0:
        raise DsgError(DSG_EINVAL, "workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")


def peel(row_ptr, col_idx, eps=(1, 10), *, m: int | None = None, extract: bool = True,
         best_ids=None, removed_at: bool | object = False, trace: bool = False, workspace=None,
         launch: dict | None = None, profile: bool = False, stream=None) -> PeelResult:
    """Peel the graph (row_ptr, col_idx) with eps = eps[0] / eps[1].

    row_ptr, col_idx: contiguous torch.int32 tensors on the current HIP device.
    m defaults to len(col_idx) // 2.  ``removed_at=True`` returns the pass in
    which each vertex failed (or pass a preallocated int32[n] tensor).
    ``workspace`` is an optional uint8 device tensor of at least
    :func:`workspace_bytes` bytes; without it the library allocates one.
    ``launch`` overrides the launch shape (``mark_grid``, ``walk_grid``,
    ``pass_batch``) and sets flags: ``bin_regions``, ``no_progress``, and
    ``id_buckets`` (True: key the degree records of every pass by neighbour
    id; False: never); results never depend on it.
    """
    import torch
    _check_int32_cuda("row_ptr", row_ptr)
    _check_int32_cuda("col_idx", col_idx)
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr needs n+1 entries")
    if m is None:
        m = col_idx.numel() // 2
    num, den = int(eps[0]), int(eps[1])
    dev = row_ptr.device
    h = lib()
    csr = CSR(row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None)
    best = None
    if extract:
        if best_ids is not None:
            _check_int32_cuda("best_ids", best_ids)
            if best_ids.numel() < n:
                raise ValueError("best_ids needs room for n ids")
            best = best_ids
        else:
            best = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    rem = None
    if removed_at is True:
        rem = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    elif removed_at is not False and removed_at is not None:
        _check_int32_cuda("removed_at", removed_at)
        if removed_at.numel() < n:
            raise ValueError("removed_at needs n entries")
        rem = removed_at
    ws_ptr, ws_len = None, 0
    if workspace is not None:
        if not workspace.is_cuda:
            raise TypeError("workspace must be device memory")
        ws_ptr, ws_len = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    cap = (n + 1) if trace else 0
    cap = min(cap, 4096)
    tr = (PassTrace * max(cap, 1))()
    ln = None
    if launch:
        ln = Launch(int(launch.get("mark_grid", 0)), int(launch.get("walk_grid", 0)),
                    int(launch.get("pass_batch", 0)),
                    (LAUNCH_BIN_REGIONS if launch.get("bin_regions") else 0)
                    | (LAUNCH_NO_PROGRESS if launch.get("no_progress") else 0)
                    | (LAUNCH_ID_BUCKETS if launch.get("id_buckets") is True else 0)
                    | (LAUNCH_NO_ID_BUCKETS if launch.get("id_buckets") is False else 0))
    prof = Profile() if profile else None
    res = Result()
    with torch.cuda.device(dev):
        rc = h.dsg_peel_ex(ctypes.byref(csr), n, m, num, den,
                           best.data_ptr() if best is not None else None,
                           rem.data_ptr() if rem is not None else None, ctypes.byref(res),
                           ctypes.addressof(tr) if cap else None, cap,
                           ctypes.byref(ln) if ln is not None else None,
                           ctypes.byref(prof) if prof is not None else None,
                           ws_ptr, ws_len, _stream_handle(stream))
    if rc != DSG_OK:
        raise DsgError(rc, "dsg_peel_ex")
    passes = []
    for k in range(min(res.passes, cap)):
        passes.append({f: int(getattr(tr[k], f)) for f in TRACE_FIELDS})
    pd = None
    if prof is not None:
        pd = {f: getattr(prof, f) for f, _ in Profile._fields_}
    return PeelResult(best=best[:res.best_size] if best is not None else None,
                      num=res.dens_num, den=res.dens_den, passes=res.passes,
                      best_pass=res.best_pass,
                      removed_at=rem[:n] if rem is not None else None, trace=passes, profile=pd)


@dataclass
class Cbds:
    best: object        # torch.int32 device tensor: S ascending (None if not extracted)
    num: int            # |E(S)|
    den: int            # |S|
    core_num: int       # |E(C_K)|
    core_den: int       # |C_K|
    K: int              # order of the densest core
    kmax: int
    passes: int
    n_eligible: int
    n_legit: int
    core: object = None  # torch.int32 device tensor of core numbers, or None
    trace: list = field(default_factory=list)


def cbds(row_ptr, col_idx, *, m: int | None = None, extract: bool = True, core: bool = False,
         trace: bool = False, workspace=None, stream=None) -> Cbds:
    """CBDS-P (Section 3.2, Algorithm 2) of the device graph: the densest
    k-core extended by legitimate vertices (dsg_cbds)."""
    import torch
    _check_int32_cuda("row_ptr", row_ptr)
    _check_int32_cuda("col_idx", col_idx)
    n = row_ptr.numel() - 1
    if m is None:
        m = col_idx.numel() // 2
    dev = row_ptr.device
    csr = CSR(row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None)
    best = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if extract else None
    cores = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if core else None
    ws_ptr, ws_len = None, 0
    if workspace is not None:
        ws_ptr, ws_len = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    cap = min(4096, 2 * n + 2) if trace else 0
    tr = (PassTrace * max(cap, 1))()
    res = CbdsResult()
    with torch.cuda.device(dev):
        rc = lib().dsg_cbds(ctypes.byref(csr), n, m,
                            best.data_ptr() if best is not None else None,
                            cores.data_ptr() if cores is not None else None, ctypes.byref(res),
                            ctypes.addressof(tr) if cap else None, cap, ws_ptr, ws_len,
                            _stream_handle(stream))
    if rc != DSG_OK:
        raise DsgError(rc, "dsg_cbds")
    passes = [{f: int(getattr(tr[k], f)) for f in TRACE_FIELDS} for k in range(min(res.passes, cap))]
    return Cbds(best=best[:res.best_size] if best is not None else None, num=res.dens_num,
                den=res.dens_den, core_num=res.core_num, core_den=res.core_den, K=res.core_k,
                kmax=res.kmax, passes=res.passes, n_eligible=res.n_eligible,
                n_legit=res.n_legit, core=cores[:n] if cores is not None else None, trace=passes)


def validate_csr(row_ptr, col_idx, m: int | None = None, stream=None) -> int:
    """0 if the device CSR meets the input contract, else the violated rule
    number (see include/dsg.h)."""
    import torch
    _check_int32_cuda("row_ptr", row_ptr)
    _check_int32_cuda("col_idx", col_idx)
    n = row_ptr.numel() - 1
    m = col_idx.numel() // 2 if m is None else m
    csr = CSR(row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None)
    detail = _I32(0)
    with torch.cuda.device(row_ptr.device):
        rc = lib().dsg_validate_csr(ctypes.byref(csr), n, m, ctypes.byref(detail),
                                    _stream_handle(stream))
    if rc == DSG_EINVAL and detail.value:
        return int(detail.value)
    if rc != DSG_OK:
        raise DsgError(rc, "dsg_validate_csr")
    return 0


# --------------------------------------------------------------------------
# batches: many graphs in one persistent launch
# --------------------------------------------------------------------------

#: int64 words per dsg_batch_result
RESULT_WORDS = ctypes.sizeof(BatchResult) // 8


def batch_workspace_bytes(count: int, entries: int, out_len: int) -> int:
    """Workspace bytes for `count` graphs with `entries` adjacency entries in
    total (sum of 2m) and out_len output slots."""
    return int(lib().dsg_batch_workspace_bytes(count, entries, out_len))


def batch_table(n, m, row_ptr_off, col_idx_off, out_off, eps):
    """ctypes array of dsg_batch_graph rows from per-graph sequences; ``eps``
    is one (num, den) pair for all graphs or a sequence of pairs."""
    count = len(n)
    tab = (BatchGraph * max(count, 1))()
    per_graph = count > 0 and isinstance(eps[0], (tuple, list))
    for i in range(count):
        num, den = eps[i] if per_graph else eps
        tab[i] = BatchGraph(int(row_ptr_off[i]), int(col_idx_off[i]), int(out_off[i]), int(n[i]),
                            int(m[i]), int(num), int(den), 0)
    return tab, count


class Batch:
    """A prepared batch: the table uploaded into a device workspace and the
    launch shape chosen (dsg_batch_prepare).  :meth:`run` enqueues the
    persistent launch and returns at once; :meth:`results` reads them."""

    def __init__(self, table, count: int, row_ptr_len: int, col_idx_len: int, out_len: int, *,
                 launch: dict | None = None, workspace=None, device=None, stream=None):
        import torch
        self.count = count
        self.out_len = out_len
        dev = torch.device(device or "cuda")
        self.entries = sum(2 * int(table[i].m) for i in range(count))
        nbytes = batch_workspace_bytes(count, self.entries, out_len)
        if nbytes == 0:
            raise DsgError(DSG_EINVAL, "dsg_batch_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.workspace = workspace
        ln = None
        if launch:
            ln = BatchLaunch(int(launch.get("block", 0)), int(launch.get("blocks_per_cu", 0)),
                             int(launch.get("grid", 0)), int(launch.get("walk_items", 0)))
        self.plan = BatchPlan()
        with torch.cuda.device(dev):
            rc = lib().dsg_batch_prepare(ctypes.addressof(table), count, row_ptr_len, col_idx_len,
                                         out_len, ctypes.byref(ln) if ln is not None else None,
                                         workspace.data_ptr(),
                                         workspace.numel() * workspace.element_size(),
                                         _stream_handle(stream), ctypes.byref(self.plan))
        if rc != DSG_OK:
            raise DsgError(rc, "dsg_batch_prepare")
        self.device = dev

    @property
    def shape(self) -> dict:
        p = self.plan
        return {"block": p.block, "blocks_per_cu": p.blocks_per_cu, "grid": p.grid,
                "walk_items": p.walk_items, "lds_bytes": p.lds_bytes,
                "lds_vertices": p.lds_vertices, "state_bits": p.state_bits}

    def run(self, row_ptr, col_idx, *, best_ids=None, removed_at=None, results=None,
            stream=None):
        """Enqueue the peel of every graph; returns the device result tensor
        (int64, count x RESULT_WORDS).  No host synchronisation."""
        import torch
        _check_int32_cuda("row_ptr", row_ptr)
        _check_int32_cuda("col_idx", col_idx)
        for name, t in (("best_ids", best_ids), ("removed_at", removed_at)):
            if t is not None:
                _check_int32_cuda(name, t)
                if t.numel() < self.out_len:
                    raise ValueError(f"{name} needs {self.out_len} entries")
        if results is None:
            results = torch.empty((max(self.count, 1), RESULT_WORDS), dtype=torch.int64,
                                  device=self.device)
        with torch.cuda.device(self.device):
            rc = lib().dsg_batch_run(ctypes.byref(self.plan), row_ptr.data_ptr(),
                                     col_idx.data_ptr(),
                                     best_ids.data_ptr() if best_ids is not None else None,
                                     removed_at.data_ptr() if removed_at is not None else None,
                                     results.data_ptr(), _stream_handle(stream))
        if rc != DSG_OK:
            raise DsgError(rc, "dsg_batch_run")
        return results

    @staticmethod
    def results(res) -> list[dict]:
        """Host list of per-graph result dicts from a device result tensor."""
        import numpy as np
        a = res.cpu().numpy().astype(np.int64)
        out = []
        for row in a:
            out.append({"num": int(row[0]), "den": int(row[1]),
                        "passes": int(np.int32(row[2] & 0xFFFFFFFF)),
                        "best_pass": int(np.int32((row[2] >> 32) & 0xFFFFFFFF)),
                        "best_size": int(row[3]),
                        "status": int(np.int32(row[4] & 0xFFFFFFFF))})
        return out


# --------------------------------------------------------------------------
# peeling without the host
# --------------------------------------------------------------------------

def peel_async(row_ptr, col_idx, eps=(1, 10), *, workspace, m: int | None = None,
               best_ids=None, removed_at=None, result=None, head_passes: int = 0,
               stream=None):
    """Enqueue dsg_peel_async: every pass runs on the device, nothing waits
    for it and nothing is allocated by the library.  Returns the device
    result tensor (int64, RESULT_WORDS words: one dsg_batch_result; read it
    with :func:`async_result` after synchronising).  ``workspace`` is a
    uint8 device tensor of at least :func:`workspace_bytes` bytes;
    ``head_passes`` > 0 sets how many passes are enqueued as kernels before
    the device loop takes over."""
    import torch
    _check_int32_cuda("row_ptr", row_ptr)
    _check_int32_cuda("col_idx", col_idx)
    n = row_ptr.numel() - 1
    if m is None:
        m = col_idx.numel() // 2
    for name, t in (("best_ids", best_ids), ("removed_at", removed_at)):
        if t is not None:
            _check_int32_cuda(name, t)
            if t.numel() < n:
                raise ValueError(f"{name} needs n entries")
    if workspace is None or not workspace.is_cuda:
        raise TypeError("peel_async needs a device workspace")
    if result is None:
        result = torch.empty(RESULT_WORDS, dtype=torch.int64, device=row_ptr.device)
    csr = CSR(row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None)
    ln = Launch(0, 0, int(head_passes), 0) if head_passes else None
    with torch.cuda.device(row_ptr.device):
        rc = lib().dsg_peel_async(ctypes.byref(csr), n, m, int(eps[0]), int(eps[1]),
                                  best_ids.data_ptr() if best_ids is not None else None,
                                  removed_at.data_ptr() if removed_at is not None else None,
                                  result.data_ptr(),
                                  ctypes.byref(ln) if ln is not None else None,
                                  workspace.data_ptr(),
                                  workspace.numel() * workspace.element_size(),
                                  _stream_handle(stream))
    if rc != DSG_OK:
        raise DsgError(rc, "dsg_peel_async")
    return result


def async_result(res) -> dict:
    """Host dict of a device result written by dsg_peel_async."""
    return Batch.results(res.reshape(1, RESULT_WORDS))[0]


# --------------------------------------------------------------------------
# the exact densest subgraph
# --------------------------------------------------------------------------

@dataclass
class Exact:
    num: int        # |E(S*)|
    den: int        # |S*|
    flows: int      # maximum flows solved
    relabels: int   # global relabels over all flows
    best: object = None  # torch.int32 device tensor: S* ascending, or None

    @property
    def density(self) -> float:
        return self.num / self.den if self.den else 0.0


def exact_density(row_ptr, col_idx, *, m: int | None = None, extract: bool = True,
                  workspace=None, stream=None) -> Exact:
    """The exact maximum density rho* of the device graph and its largest
    densest subgraph S* (dsg_exact_density: Goldberg's construction with a
    device push-relabel flow inside Dinkelbach's iteration)."""
    import torch
    _check_int32_cuda("row_ptr", row_ptr)
    _check_int32_cuda("col_idx", col_idx)
    n = row_ptr.numel() - 1
    if m is None:
        m = col_idx.numel() // 2
    dev = row_ptr.device
    best = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if extract else None
    ws_ptr, ws_len = None, 0
    if workspace is not None:
        ws_ptr, ws_len = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    csr = CSR(row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None)
    res = ExactResult()
    with torch.cuda.device(dev):
        rc = lib().dsg_exact_density(ctypes.byref(csr), n, m,
                                     best.data_ptr() if best is not None else None,
                                     ctypes.byref(res), ws_ptr, ws_len, _stream_handle(stream))
    if rc != DSG_OK:
        raise DsgError(rc, "dsg_exact_density")
    return Exact(num=res.dens_num, den=res.dens_den, flows=res.flows, relabels=res.relabels,
                 best=best[:res.set_size] if best is not None else None)
