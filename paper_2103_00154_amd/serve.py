"""Serving loop: peel requests that arrive over time, batched as they come.

A request is one graph (CSR in pinned host memory) and one eps.  The server
owns one device arena - its HBM budget - and admits waiting requests in
arrival order while their footprint fits: the graph's CSR, its output slots
and its share of the batch workspace (dsg_batch_workspace_bytes).  Admitted
requests are uploaded into the arena, where the CSR stays resident until the
request completes, and are peeled by the persistent batch kernel
(dsg_batch_run) as one micro-batch on one of several HIP streams.  Requests
that arrive while earlier micro-batches are still on the device are admitted
as soon as a stream and memory are free, so their work overlaps on the device
with the batches already running (continuous batching).  Completed batches
free their memory, and their results are read back.

Graphs with more vertices than a workgroup keeps in LDS would hold one CU
for a long time (their state spills to device memory), so they take a
separate lane instead: each is peeled by the single-graph path without the
host (dsg_peel_async: every pass enqueued at once, the pass loop on the
device), which spreads one graph over the whole device, on one of several
lane streams, concurrently with the batches.  The serving thread enqueues a
large request and moves on; an event tells when its result has arrived.

Under a load beyond capacity the server can shed work: with ``max_queue_s``
set, a request still waiting that long after its arrival is rejected
(``Request.rejected``) instead of being admitted, so the requests that are
served keep a bounded latency and the served rate stays at capacity.

Every result is exactly the result of peeling the graph alone: the kernels
are exact integer code, and in a batch a graph is peeled by one workgroup,
independently of what else shares the launch.
"""
from __future__ import annotations

import bisect
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import dsg

ALIGN = 256


class Arena:
    """First-fit allocator over [0, size) bytes, 256-byte granules; host-side
    bookkeeping for one device buffer."""

    def __init__(self, size: int):
        self.size = size - size % ALIGN
        self._free = [(0, self.size)]  # sorted (offset, length)
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes: int) -> int | None:
        need = max(ALIGN, (nbytes + ALIGN - 1) // ALIGN * ALIGN)
        for i, (off, ln) in enumerate(self._free):
            if ln >= need:
                if ln == need:
                    del self._free[i]
                else:
                    self._free[i] = (off + need, ln - need)
                self.used += need
                self.peak = max(self.peak, self.used)
                return off
        return None

    def free(self, off: int, nbytes: int) -> None:
        ln = max(ALIGN, (nbytes + ALIGN - 1) // ALIGN * ALIGN)
        i = bisect.bisect_left(self._free, (off, 0))
        self._free.insert(i, (off, ln))
        self.used -= ln
        # coalesce with the neighbours
        if i + 1 < len(self._free) and off + ln == self._free[i + 1][0]:
            self._free[i] = (off, ln + self._free[i + 1][1])
            del self._free[i + 1]
        if i > 0 and self._free[i - 1][0] + self._free[i - 1][1] == off:
            po, pl = self._free[i - 1]
            self._free[i - 1] = (po, pl + self._free[i][1])
            del self._free[i]

    def largest_free(self) -> int:
        return max((ln for _, ln in self._free), default=0)


@dataclass
class HostGraph:
    """A request graph in pinned host memory: row_ptr (n+1) then col_idx (2m)."""

    n: int
    m: int
    csr: object  # pinned torch.int32 tensor of n + 1 + 2m entries

    @staticmethod
    def from_graph(g) -> "HostGraph":
        import torch
        buf = np.empty(g.n + 1 + 2 * g.m, dtype=np.int32)
        buf[:g.n + 1] = g.row_ptr
        buf[g.n + 1:] = g.col_idx[:2 * g.m]
        return HostGraph(g.n, g.m, torch.from_numpy(buf).pin_memory())


@dataclass
class Request:
    rid: int
    graph: HostGraph
    eps: tuple
    arrival: float                # seconds since the start of the run
    admitted: float = -1.0
    done: float = -1.0
    result: dict | None = None
    best: np.ndarray | None = None
    rejected: bool = False


@dataclass
class _LaneJob:
    req: Request
    stream: object
    event: object
    allocs: list                  # (offset, bytes) in the arena
    res_host: object              # pinned copy of the device result
    best_host: object             # pinned copy of the best-id slots


@dataclass
class _MicroBatch:
    reqs: list
    stream: object
    event: object
    allocs: list                  # (offset, bytes) in the arena
    res_host: object
    best_host: object
    best_off: list = field(default_factory=list)
    res_dev: object = None
    solo: bool = False


def footprint(n: int, m: int) -> int:
    """Arena bytes one request holds while admitted: its CSR, its output
    slots and its part of the batch workspace (per-vertex arrays, table row
    and tile table), each rounded to the arena granule."""
    def r(x):
        return (x + ALIGN - 1) // ALIGN * ALIGN
    return r(4 * (n + 1 + 2 * m)) + r(4 * n) + 24 * n + 72 + 4 * (2 * m // 256 + 2) + 6 * ALIGN


class Server:
    """Continuous-batching peel server on one device (see the module doc).

    ``big_vertices``: requests with more vertices go to the single-graph lane
    (None: the LDS vertex capacity of the batch kernel's launch shape; 0 or a
    huge value disables the lane); ``big_lanes`` lane streams carry them.
    ``reserve_cus``: CUs kept free of batch workgroups for the single-graph
    lane (None: a quarter of the CUs while the lane is on).  A persistent
    batch workgroup holds most of its CU's LDS, so without a reserve a loaded
    server leaves the lane's kernels no CU to run on; each micro-batch's grid
    is capped at (CUs - reserve) / streams workgroups.
    ``overflow``: when the lane has a backlog (twice as many requests waiting
    as it has streams), a large request goes to the batch kernel instead, in
    a micro-batch of its own.
    ``max_queue_s``: shed load - a request not admitted within this many
    seconds of its arrival is rejected (None: every request waits its turn).
    """

    def __init__(self, budget_bytes: int, *, streams: int = 4, max_batch: int = 512,
                 launch: dict | None = None, device=None, big_vertices: int | None = None,
                 big_lanes: int = 4, reserve_cus: int | None = None, overflow: bool = False,
                 max_queue_s: float | None = None):
        import torch
        self.device = torch.device(device or "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.buf = torch.empty(budget_bytes, dtype=torch.uint8, device=self.device)
        self.arena = Arena(budget_bytes)
        if big_vertices is None:
            big_vertices = _lds_vertices(launch, self.device)
        self.big_vertices = big_vertices
        cus = torch.cuda.get_device_properties(self.device).multi_processor_count
        if reserve_cus is None:
            reserve_cus = cus // 4 if big_vertices else 0
        self.batch_grid = max(1, (cus - min(reserve_cus, cus - 1)) // max(streams, 1))
        self.big_waiting: deque[Request] = deque()
        self.big_done = 0
        self.error: BaseException | None = None
        nl = big_lanes if big_vertices else 0
        self.lane_streams = [torch.cuda.Stream(device=self.device) for _ in range(nl)]
        self.lane_busy: list = [None] * nl
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.busy = [None] * streams
        self.waiting: deque[Request] = deque()
        self.solo: deque[Request] = deque()   # large requests overflowing into batches
        self.overflow = overflow
        self.overflowed = 0
        self.max_queue_s = max_queue_s
        self.rejected = 0
        self.max_batch = max_batch
        self.launch = launch
        self.completed: list[Request] = []
        self.batches = 0
        self.batch_sizes: list[int] = []
        self.max_in_flight = 0
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> None:
        big = bool(self.big_vertices) and req.graph.n > self.big_vertices
        need = (_single_footprint(req.graph.n, req.graph.m) if big
                else footprint(req.graph.n, req.graph.m))
        if need > self.arena.size:
            raise ValueError(f"request {req.rid} needs more memory than the whole budget")
        if big:
            backlog = len(self.big_waiting) >= 2 * max(len(self.lane_streams), 1)
            if (self.overflow and backlog and
                    footprint(req.graph.n, req.graph.m) <= self.arena.size):
                self.solo.append(req)
                self.overflowed += 1
            else:
                self.big_waiting.append(req)
        else:
            self.waiting.append(req)

    @property
    def idle(self) -> bool:
        return (not self.big_waiting and not self.waiting and not self.solo
                and all(b is None for b in self.busy)
                and all(j is None for j in self.lane_busy))

    def close(self) -> None:
        """Nothing runs in the background; kept for callers that close."""

    # ------------------------------------------------------------------
    def _reap(self) -> None:
        for k, mb in enumerate(self.busy):
            if mb is None or not mb.event.query():
                continue
            t = self.now()
            results = dsg.Batch.results(mb.res_host)
            best = mb.best_host.numpy()
            for i, rq in enumerate(mb.reqs):
                rq.done = t
                rq.result = results[i]
                a = mb.best_off[i]
                rq.best = best[a:a + rq.result["best_size"]].copy()
            for off, nb in mb.allocs:
                self.arena.free(off, nb)
            self.completed.extend(mb.reqs)
            self.busy[k] = None
        for k, job in enumerate(self.lane_busy):
            if job is None or not job.event.query():
                continue
            rq = job.req
            rq.done = self.now()
            rq.result = dsg.Batch.results(job.res_host)[0]
            rq.best = job.best_host.numpy()[:rq.result["best_size"]].copy()
            for off, nb in job.allocs:
                self.arena.free(off, nb)
            self.completed.append(rq)
            self.big_done += 1
            self.lane_busy[k] = None

    def _shed(self) -> None:
        """Reject the requests that have waited longer than max_queue_s."""
        if self.max_queue_s is None:
            return
        now = self.now()
        for q in (self.waiting, self.big_waiting, self.solo):
            while q and now - q[0].arrival > self.max_queue_s:
                rq = q.popleft()
                rq.rejected = True
                rq.done = now
                self.rejected += 1
                self.completed.append(rq)

    def _shared_bytes(self, take) -> tuple[int, int]:
        sum_n = sum(r.graph.n for r in take)
        sum_e = sum(2 * r.graph.m for r in take)
        return dsg.batch_workspace_bytes(len(take), sum_e, sum_n), 4 * max(sum_n, 1)

    def _try_place(self, sizes) -> list | None:
        got = []
        for nb in sizes:
            off = self.arena.alloc(nb)
            if off is None:
                for o, b in got:
                    self.arena.free(o, b)
                return None
            got.append((off, nb))
        return got

    def _launch_lane(self, k: int) -> bool:
        """Enqueue the head large request on lane stream k (upload, device
        peel, result copies, event); False if its memory is not free yet."""
        import torch
        rq = self.big_waiting[0]
        g = rq.graph
        nb_csr = 4 * (g.n + 1 + 2 * g.m)
        nb_ws = dsg.workspace_bytes(g.n, g.m)
        got = self._try_place((nb_csr, 4 * max(g.n, 1), nb_ws))
        if got is None:
            return False
        self.big_waiting.popleft()
        rq.admitted = self.now()
        (o_csr, _), (o_best, _), (o_ws, _) = got
        ints = self.buf.view(torch.int32)
        s = self.lane_streams[k]
        with torch.cuda.stream(s):
            dev = ints[o_csr // 4:o_csr // 4 + g.csr.numel()]
            dev.copy_(g.csr, non_blocking=True)
            best = ints[o_best // 4:o_best // 4 + max(g.n, 1)]
            res = torch.empty(dsg.RESULT_WORDS, dtype=torch.int64, device=self.device)
            dsg.peel_async(dev[:g.n + 1], dev[g.n + 1:] if g.m else dev[:1], rq.eps, m=g.m,
                           workspace=self.buf[o_ws:o_ws + nb_ws], best_ids=best, result=res,
                           stream=s)
            res_host = torch.empty(dsg.RESULT_WORDS, dtype=torch.int64, pin_memory=True)
            res_host.copy_(res, non_blocking=True)
            best_host = torch.empty(best.numel(), dtype=torch.int32, pin_memory=True)
            best_host.copy_(best, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self.lane_busy[k] = _LaneJob(rq, s, ev, got, res_host.view(1, -1), best_host)
        return True

    def _launch(self, k: int, queue=None) -> None:
        self._launch_locked(k, self.waiting if queue is None else queue,
                            self.max_batch if queue is None else 1)
    def _launch_locked(self, k: int, queue, max_batch: int) -> None:
        import torch
        take, allocs = [], []
        # admit in arrival order while the request's CSR and the batch's
        # shared regions (workspace, output slots) fit; the head request
        # waits for memory when it does not
        while queue and len(take) < max_batch:
            rq = queue[0]
            nb = 4 * (rq.graph.n + 1 + 2 * rq.graph.m)
            off = self.arena.alloc(nb)
            if off is None:
                break
            trial = self._try_place(self._shared_bytes(take + [rq]))
            if trial is None:
                self.arena.free(off, nb)
                break
            for o, b in trial:
                self.arena.free(o, b)
            allocs.append((off, nb))
            take.append(queue.popleft())
        if not take:
            return
        csr_off = [o for o, _ in allocs]
        sum_n = sum(r.graph.n for r in take)
        ws_bytes, best_bytes = self._shared_bytes(take)
        (ws_off, _), (best_off, _) = self._try_place((ws_bytes, best_bytes))
        allocs += [(ws_off, ws_bytes), (best_off, best_bytes)]
        now = self.now()
        for rq in take:
            rq.admitted = now
        s = self.streams[k]
        ints = self.buf.view(torch.int32)
        n_arr = [r.graph.n for r in take]
        m_arr = [r.graph.m for r in take]
        rp_off = [o // 4 for o in csr_off]
        ci_off = [o // 4 + r.graph.n + 1 for o, r in zip(csr_off, take)]
        out = np.zeros(len(take), dtype=np.int64)
        if len(take) > 1:
            out[1:] = np.cumsum(n_arr)[:-1]
        eps = [r.eps for r in take]
        tab, count = dsg.batch_table(n_arr, m_arr, rp_off, ci_off, out, eps)
        ws = self.buf[ws_off:ws_off + ws_bytes]
        with torch.cuda.stream(s):
            launch = dict(self.launch or {})
            launch["grid"] = min(count, self.batch_grid)
            plan = dsg.Batch(tab, count, ints.numel(), ints.numel(), sum_n, launch=launch,
                             workspace=ws, device=self.device, stream=s)
            for o, r in zip(csr_off, take):
                ints[o // 4:o // 4 + r.graph.csr.numel()].copy_(r.graph.csr, non_blocking=True)
            best = ints[best_off // 4:best_off // 4 + max(sum_n, 1)]
            res = torch.empty((count, dsg.RESULT_WORDS), dtype=torch.int64, device=self.device)
            plan.run(ints, ints, best_ids=best, results=res, stream=s)
            res_host = torch.empty(res.shape, dtype=torch.int64, pin_memory=True)
            res_host.copy_(res, non_blocking=True)
            best_host = torch.empty(best.numel(), dtype=torch.int32, pin_memory=True)
            best_host.copy_(best, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self.busy[k] = _MicroBatch(take, s, ev, allocs, res_host, best_host, list(out), res,
                                   solo=max_batch == 1)
        self.batches += 1
        self.batch_sizes.append(len(take))
        self.max_in_flight = max(self.max_in_flight, sum(b is not None for b in self.busy))

    def tick(self) -> None:
        """Reap finished work, shed requests waiting too long, then launch
        large requests on free lane streams and micro-batches on free batch
        streams."""
        self._reap()
        self._shed()
        for k in range(len(self.lane_busy)):
            if self.lane_busy[k] is None and self.big_waiting:
                if not self._launch_lane(k):
                    break
        # overflowing large requests use at most half of the streams
        solo_cap = max(1, len(self.busy) // 2)
        for k in range(len(self.busy)):
            if self.busy[k] is not None:
                continue
            solo_now = sum(1 for b in self.busy if b is not None and b.solo)
            if self.solo and solo_now < solo_cap:
                self._launch(k, self.solo)
            elif self.waiting:
                self._launch(k)

    def drain(self, timeout_s: float = 120.0) -> None:
        end = time.perf_counter() + timeout_s
        while not self.idle:
            if time.perf_counter() > end:
                raise TimeoutError("server did not drain")
            self.tick()


def _single_footprint(n: int, m: int) -> int:
    """Arena bytes of a request in the single-graph lane: CSR, output slots
    and the dsg_peel workspace."""
    def r(x):
        return (x + ALIGN - 1) // ALIGN * ALIGN
    return r(4 * (n + 1 + 2 * m)) + r(4 * max(n, 1)) + r(dsg.workspace_bytes(n, m))


_LDS_CACHE: dict = {}


def _lds_vertices(launch, device) -> int:
    """Vertices per graph the batch kernel keeps in LDS for this shape."""
    key = (str(device), tuple(sorted((launch or {}).items())))
    if key not in _LDS_CACHE:
        import torch
        tab, count = dsg.batch_table([1], [0], [0], [0], [0], (1, 10))
        ws = torch.empty(dsg.batch_workspace_bytes(1, 0, 1), dtype=torch.uint8, device=device)
        b = dsg.Batch(tab, count, 2, 0, 1, launch=launch, workspace=ws, device=device)
        _LDS_CACHE[key] = b.shape["lds_vertices"]
    return _LDS_CACHE[key]


def poisson_arrivals(count: int, qps: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process of rate qps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


def run_load(server: Server, graphs: list, eps_choices, qps: float, count: int,
             seed: int = 0, timeout_s: float = 300.0) -> list[Request]:
    """Offer `count` requests at Poisson rate `qps`; request i peels
    graphs[i % len(graphs)] with an eps drawn from eps_choices.  Returns the
    completed requests (arrival, admission, completion times in seconds)."""
    rng = np.random.default_rng(seed + 1)
    arrivals = poisson_arrivals(count, qps, seed)
    pick = rng.integers(0, len(eps_choices), size=count)
    reqs = [Request(i, graphs[i % len(graphs)], tuple(eps_choices[pick[i]]), float(arrivals[i]))
            for i in range(count)]
    server.t0 = time.perf_counter()
    nxt = 0
    while nxt < count or not server.idle:
        if server.now() > arrivals[-1] + timeout_s:
            raise TimeoutError(f"{count - len(server.completed)} requests still open")
        now = server.now()
        while nxt < count and reqs[nxt].arrival <= now:
            server.submit(reqs[nxt])
            nxt += 1
        server.tick()
    return reqs


def latency_stats(reqs: list[Request]) -> dict:
    """Latency of the served requests (arrival to host-visible result), the
    rate they were served at over the run, and how many were rejected."""
    served = [r for r in reqs if not r.rejected]
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    out = {"requests": len(reqs), "served": len(served), "rejected": len(reqs) - len(served),
           "graphs_per_s": round(len(served) / span, 1)}
    if served:
        lat = np.array([r.done - r.arrival for r in served]) * 1e3
        queue = np.array([r.admitted - r.arrival for r in served]) * 1e3
        out.update({"p50_ms": round(float(np.percentile(lat, 50)), 3),
                    "p99_ms": round(float(np.percentile(lat, 99)), 3),
                    "mean_ms": round(float(lat.mean()), 3),
                    "queue_p50_ms": round(float(np.percentile(queue, 50)), 3)})
    return out
