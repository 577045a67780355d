#!/usr/bin/env python3
"""Throughput of Bahmani (2+2eps) peeling on one MI355X.

One step = one complete peel of the workload graph (init, every pass's mark
and neighbour walk, extraction of S~), with the CSR already resident in HBM.
The metric is peeled edges per second, GTEPS = m / t_step, next to the
fraction of the HBM roofline that the dominant kernel (the neighbour walk)
reaches, and the CPU oracle timed on the host's cores.

Default workload: R-MAT scale 24 (n = 16,777,216), edge factor 16,
(a,b,c,d) = (.57,.19,.19,.05), seed 0, plus a planted G(2000, 1/2) block on
random ids (seed 1), eps = 1/10 - the largest single-graph configuration.

The same line carries the batched half of the metric under "batch": 4096
graphs (n log-uniform in [100, 100000], alternating Erdos-Renyi and
Chung-Lu with exponent in [2.1, 2.8], average degree in [4, 64], eps = 1/10)
peeled in one persistent launch with an autotuned shape, as graphs/s next to
the same graphs peeled one call (one graph) at a time.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib

import numpy as np
import json
import os
import statistics
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

METRIC = "peeled edges/sec (GTEPS) + % HBM roofline; batched graphs/sec vs 1-graph/launch"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = ROOT / "profiles" / "walk_traffic_rmat24.json"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str):
    from paper_2103_00154_amd import inputs
    if name == "rmat24":
        g = inputs.rmat(24, 16, seed=0, planted=(2000, 0.5, 1))
        desc = ("R-MAT scale 24, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed 0, "
                "planted G(2000,1/2) on random ids (seed 1)")
    elif name == "rmat20":
        g = inputs.rmat(20, 16, seed=0)
        desc = "R-MAT scale 20, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed 0"
    elif name == "er10k":
        g = inputs.erdos_renyi(10_000, 50_000, 0)
        desc = "Erdos-Renyi n=10000 m=50000, seed 0"
    else:
        raise SystemExit(f"unknown workload {name}")
    return g, desc


def kernel_source_digest() -> str:
    """Digest of the sources the single-graph kernels are built from (the
    traffic record is valid only for these exact sources)."""
    h = hashlib.sha256()
    for name in ("common.h", "peel.hip"):
        h.update((ROOT / "paper_2103_00154_amd" / "csrc" / name).read_bytes())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, launches: int):
    """HBM bytes per walk launch measured with rocprofv3 counters, if they
    were taken on the current kernel source."""
    if not TRAFFIC_FILE.exists():
        return None
    try:
        rec = json.loads(TRAFFIC_FILE.read_text())
    except ValueError:
        return None
    if rec.get("kernel_digest") != kernel_source_digest() or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


def measure_stream(nbytes: int = 4 << 30, reps: int = 5) -> dict:
    """The hand-written STREAM kernels (measure/stream.hip) on this GPU:
    copy (b = a) and triad (c = a + 3 b) over int32 arrays of `nbytes`
    bytes each; median GB/s of bytes read plus written."""
    import ctypes
    from paper_2103_00154_amd import _build
    lib = ctypes.CDLL(str(_build.ensure_stream()))
    lib.stream_measure.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    lib.stream_measure.restype = ctypes.c_int
    best = None
    for bpc in (4, 8, 16):
        c, t = ctypes.c_double(0), ctypes.c_double(0)
        rc = lib.stream_measure(nbytes, reps, bpc, ctypes.byref(c), ctypes.byref(t))
        if rc != 0:
            raise RuntimeError(f"stream_measure failed with HIP error {rc}")
        log(f"STREAM kernels, {bpc} workgroups per CU: copy {c.value:.0f} GB/s, "
            f"triad {t.value:.0f} GB/s")
        if best is None or c.value > best["copy"]:
            best = {"copy": c.value, "triad": t.value, "blocks_per_cu": bpc}
    return best


def measure_gather(n_ids: int, lookups: int = 1 << 27, reps: int = 5) -> dict:
    """The walk's lookup ceiling on this GPU (measure/stream.hip): uniformly
    random ids below the next power of two of `n_ids`, each read once and
    used for one 8-byte gather from a table of one word per 32 ids (the
    rank directory's shape); median billions of lookups per second."""
    import ctypes
    from paper_2103_00154_amd import _build
    lib = ctypes.CDLL(str(_build.ensure_stream()))
    lib.gather_measure.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_double)]
    lib.gather_measure.restype = ctypes.c_int
    lg = min(30, max(5, (max(n_ids, 2) - 1).bit_length()))
    best = None
    for bpc in (4, 8):
        v = ctypes.c_double(0)
        rc = lib.gather_measure(lookups, lg, reps, bpc, ctypes.byref(v))
        if rc != 0:
            raise RuntimeError(f"gather_measure failed with HIP error {rc}")
        log(f"gather probe, {bpc} workgroups per CU: {v.value:.1f} G lookups/s "
            f"({lookups} random ids below 2^{lg}, table {(1 << lg) // 32 * 8} B)")
        if best is None or v.value > best["glookups_per_s"]:
            best = {"glookups_per_s": round(v.value, 1), "lookups": lookups, "ids": 1 << lg,
                    "table_bytes": (1 << lg) // 32 * 8, "blocks_per_cu": bpc}
    return best


def host_cpu() -> dict:
    """The host's logical CPUs (usable by this process) and CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": usable, "cpu_model": model}


def measure_copy_gbs(torch, dev, nbytes: int = 4 << 30, reps: int = 5) -> float:
    """Measured copy ceiling of this GPU: a device-to-device copy of `nbytes`
    (hipMemcpyAsync), bytes read plus bytes written per second, median of
    `reps` copies timed with HIP events."""
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        z.record()
        z.synchronize()
        times.append(a.elapsed_time(z))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (statistics.median(times) * 1e-3) / 1e9


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat24", choices=["rmat24", "rmat20", "er10k"])
    ap.add_argument("--eps", default="1/10")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="single,batch,serve,sweep,cbds",
                    help="comma list of measurements to run: single (the headline "
                         "single-graph peel), batch, serve; profiler runs pick one")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched (4096-graph) measurement")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--batch-shape", default="",
                    help="BLOCK,WALK_ITEMS,BLOCKS_PER_CU instead of autotuning")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving (Poisson request stream) measurement")
    ap.add_argument("--serve-qps", default="2000,5000,10000,20000",
                    help="comma list of offered request rates for the load curve")
    ap.add_argument("--serve-requests", type=int, default=3000)
    ap.add_argument("--serve-pool", type=int, default=256)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES bytes device-to-device once (reference kernel for "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE scaling) and exit")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        src = torch.ones(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.calibrate_copy} bytes")
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} (WORLD_SIZE {world}) is not "
              "supported: the library peels one graph on a single MI355X (how the peel would "
              "shard over several GPUs is described in the design notes, not implemented).",
              file=sys.stderr)
        return 2

    num, den = (int(x) for x in args.eps.split("/"))
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 1
    from paper_2103_00154_amd import dsg

    legs = set(args.legs.split(","))
    if args.no_batch:
        legs.discard("batch")
    if args.no_serve:
        legs.discard("serve")
    if "single" not in legs:
        # profiler runs of one leg: the JSON line carries only that leg
        torch.cuda.set_device(0)
        line = {"metric": METRIC, "value": None, "unit": "GTEPS", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "legs": sorted(legs),
                "batch": bench_batch(args, torch, dsg, num, den,
                                     run_oracle=not args.no_cpu_baseline)
                if "batch" in legs else None,
                "serving": bench_serve(args, torch) if "serve" in legs else None,
                "eps_sweep": bench_sweep(args, torch, run_oracle=not args.no_cpu_baseline)
                if "sweep" in legs else None,
                "cbds": bench_cbds(args, torch, run_oracle=not args.no_cpu_baseline)
                if "cbds" in legs else None}
        print(json.dumps(line), flush=True)
        return 0

    t0 = time.time()
    g, desc = make_workload(args.workload)
    log(f"workload {args.workload}: n={g.n} m={g.m} generated in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    ws = dsg.alloc_workspace(g.n, g.m, dev)
    best = torch.empty(g.n, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        r = dsg.peel(rp, ci, (num, den), best_ids=best, workspace=ws)
    torch.cuda.synchronize()

    # timed region: whole peels, no instrumentation
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        r = dsg.peel(rp, ci, (num, den), best_ids=best, workspace=ws)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    gteps = g.m / (ms_per_step * 1e-3) / 1e9

    # the same peel through dsg_peel_async (every pass enqueued up front,
    # the loop on the device, no host synchronisation): K peels back to back
    res_async = torch.empty(dsg.RESULT_WORDS, dtype=torch.int64, device=dev)
    for _ in range(args.warmup):
        dsg.peel_async(rp, ci, (num, den), workspace=ws, best_ids=best, result=res_async)
    torch.cuda.synchronize()
    a_start = time.perf_counter()
    for _ in range(args.steps):
        dsg.peel_async(rp, ci, (num, den), workspace=ws, best_ids=best, result=res_async)
    torch.cuda.synchronize()
    ms_async = (time.perf_counter() - a_start) * 1e3 / args.steps
    ra = dsg.async_result(res_async)
    async_same = (ra["status"], ra["passes"], ra["best_pass"], ra["num"], ra["den"]) == (
        0, r.passes, r.best_pass, r.num, r.den)
    log(f"dsg_peel_async: {ms_async:.3f} ms/peel ({g.m / (ms_async * 1e-3) / 1e9:.1f} GTEPS), "
        f"result {'equal to' if async_same else 'DIFFERENT from'} dsg_peel's")

    # the same steps again with HIP events around every launch (on the
    # library's stream) for per-kernel durations
    walk_ms = apply_ms = mark_ms = 0.0
    walk_launches = 0
    walked = cross = walk_list = live = 0
    torch.cuda.synchronize()
    p_start = time.perf_counter()
    for _ in range(args.steps):
        r = dsg.peel(rp, ci, (num, den), best_ids=best, workspace=ws, profile=True)
        p = r.profile
        walk_ms += p["ms_walk"]
        apply_ms += p["ms_apply"]
        mark_ms += p["ms_mark"]
        walk_launches += p["launches_walk"]
        walked += p["walked"]
        cross += p["cross"]
        walk_list += p["walk_list"]
        live += p["live_scanned"]
    torch.cuda.synchronize()
    ms_profiled = (time.perf_counter() - p_start) * 1e3 / args.steps
    log(f"GPU: {ms_per_step:.3f} ms/step, {gteps:.1f} GTEPS, passes={r.passes} "
        f"best={r.num}/{r.den} (pass {r.best_pass}); instrumented {ms_profiled:.3f} ms/step: "
        f"walk {walk_ms / args.steps:.3f} ms, apply {apply_ms / args.steps:.3f} ms, "
        f"mark {mark_ms / args.steps:.3f} ms")

    # neighbour walk (the dominant kernel; one walk launch per pass, k_walk
    # or, in passes that key their records by neighbour id, k_walk_ids):
    # algorithmic bytes = 4 B column id + 4 B neighbour state per walked
    # entry (the method's own data); the design's intermediates are reported
    # apart as overhead, not counted as algorithmic (below)
    walk_bytes = 8 * walked
    per_launch_bytes = walk_bytes / walk_launches
    per_launch_ms = walk_ms / walk_launches
    achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
    traffic = stored_traffic(args.workload, walk_launches // args.steps)
    # whole path per step, the method's algorithmic bytes: 4 B column id +
    # 4 B neighbour state per adjacency entry (every row is read once over a
    # peel: 2m entries), 8 B per degree decrement (read-modify-write of the
    # counter), 12 B per live-list test (id, degree, re-write) and 24 B per
    # vertex (row_ptr pair, removal pass, failure list, init degree,
    # extraction read)
    path_bytes = 8 * 2 * g.m + (8 * cross + 12 * live) / args.steps + 24 * g.n
    path_gbs = path_bytes / (ms_per_step * 1e-3) / 1e9
    copy_gbs = measure_copy_gbs(torch, dev)
    log(f"device-to-device copy (runtime): {copy_gbs:.0f} GB/s (bytes read + written)")
    stream = measure_stream()
    gather = measure_gather(g.n)
    # the per-pass trace of one more (untimed) peel
    rt = dsg.peel(rp, ci, (num, den), best_ids=best, workspace=ws, trace=True)
    trace_keys = ("s_in", "e_in", "thresh", "removed", "walked", "cross", "intra", "s_out", "e_out")
    pass_trace = [{k: int(t[k]) for k in trace_keys} for t in rt.trace]
    log("pass |S_in| T |A| walked cross intra |E_out|")
    for k, t in enumerate(pass_trace):
        log(f"{k + 1} {t['s_in']} {t['thresh']} {t['removed']} {t['walked']} {t['cross']} "
            f"{t['intra']} {t['e_out']}")
    # the design's intermediates per walk launch: a 2 B record per degree
    # decrement (per walked entry in a pass that keys its records by
    # neighbour id: more than 65,536 survivors, at least 2^25 walked entries,
    # at most 2^25 vertices) and 12 B per walk-list row (row start, prefix
    # offset, owner)
    records = sum(t["walked"] if t["s_out"] > 65536 and t["walked"] >= 1 << 25
                  and g.n <= 1 << 25 else t["cross"] for t in pass_trace)
    overhead = 2 * records * args.steps + 12 * walk_list

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        times = []
        o = None
        for _ in range(args.cpu_reps):
            c0 = time.perf_counter()
            o = oracle.peel_graph(g, num, den, trace=True)
            times.append(time.perf_counter() - c0)
        t_cpu = statistics.median(times)
        cpu = dict({"value": round(g.m / t_cpu / 1e9, 4), "unit": "GTEPS", "cores": 1,
                    "kind": "oracle",
                    "sample": f"whole workload (n={g.n}, m={g.m}), single-threaded C oracle, "
                              f"median of {args.cpu_reps} runs, {t_cpu:.2f} s each"},
                   **host_cpu())
        same = ((r.passes, r.best_pass, r.num, r.den) == (o.passes, o.best_pass, o.num, o.den)
                and bool((best[:r.den].cpu().numpy() == o.best).all()))
        # the per-pass trace too (the thresholds are clamped to int32 on the GPU)
        same = same and len(pass_trace) == len(o.trace) and all(
            all(a[k] == b[k] for k in ("s_in", "e_in", "removed", "cross", "intra", "s_out",
                                       "e_out")) and a["thresh"] == min(b["thresh"], 2**31 - 1)
            for a, b in zip(pass_trace, o.trace))
        parity = "exact" if same else "MISMATCH"
        log(f"oracle: {t_cpu:.2f} s ({g.m / t_cpu / 1e9:.3f} GTEPS), parity {parity}")

    batch = None
    if "batch" in legs:
        batch = bench_batch(args, torch, dsg, num, den, run_oracle=not args.no_cpu_baseline)
    serving = None
    if "serve" in legs:
        serving = bench_serve(args, torch)
    eps_sweep = None
    if "sweep" in legs:
        eps_sweep = bench_sweep(args, torch, run_oracle=not args.no_cpu_baseline)
    cbds = None
    if "cbds" in legs:
        cbds = bench_cbds(args, torch, run_oracle=not args.no_cpu_baseline)

    line = {
        "metric": METRIC,
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}, eps={num}/{den}", "n": g.n,
                   "m": g.m, "eps": f"{num}/{den}", "passes": r.passes,
                   "launch": "library default", "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_walk / k_walk_ids (the walk of each pass)",
                     "launches_per_step": walk_launches // args.steps,
                     "ms_per_launch": round(per_launch_ms, 4),
                     "alg_bytes_per_launch": int(per_launch_bytes),
                     "alg_bytes_rule": "8 B per walked adjacency entry (column id + neighbour state)",
                     "overhead_bytes_per_launch": int(overhead / walk_launches),
                     "stream_copy": round(stream["copy"], 1),
                     "stream_triad": round(stream["triad"], 1),
                     "runtime_copy": round(copy_gbs, 1),
                     "frac_of_stream_copy": round(achieved / stream["copy"], 4),
                     "walk_gentries_per_s": round(walked / (walk_ms * 1e-3) / 1e9, 1),
                     "gather_ceiling": gather},
        "kernel_ms_per_step": {"instrumented_step": round(ms_profiled, 4),
                               "walk": round(walk_ms / args.steps, 4),
                               "apply": round(apply_ms / args.steps, 4),
                               "mark": round(mark_ms / args.steps, 4)},
        "path_roofline": {"achieved": round(path_gbs, 1), "unit": "GB/s",
                          "frac": round(path_gbs / HBM_PEAK_GBS, 4),
                          "alg_bytes_per_step": int(path_bytes),
                          "alg_bytes_rule": "8 B x 2m + 8 B x sum cross + 12 B x sum |S_in| "
                                            "+ 24 B x n"},
        "cpu_baseline": cpu,
        "parity": parity,
        "async": {"entry": "dsg_peel_async", "ms_per_step": round(ms_async, 4),
                  "gteps": round(g.m / (ms_async * 1e-3) / 1e9, 3),
                  "same_as_dsg_peel": async_same},
        "pass_trace": pass_trace,
        "batch": batch,
        "serving": serving,
        "eps_sweep": eps_sweep,
        "cbds": cbds,
    }
    print(json.dumps(line), flush=True)
    ok = parity in (None, "exact") and (batch is None or batch["parity"] in (None, "exact"))
    ok = ok and async_same
    ok = ok and (serving is None or serving["parity"] == "exact")
    ok = ok and (eps_sweep is None or eps_sweep["parity"] in (None, "exact"))
    ok = ok and (cbds is None or all(c["parity"] in (None, "exact") for c in cbds["runs"]))
    return 0 if ok else 3


def bench_batch(args, torch, dsg, num: int, den: int, run_oracle: bool) -> dict:
    """Graphs/s of one persistent launch over the whole batch vs the same
    graphs peeled by one dsg_peel call each, on the same device arrays."""
    from paper_2103_00154_amd import autotune, inputs
    t0 = time.time()
    specs = inputs.batch_specs(args.batch_count, seed=0)
    b = inputs.make_batch(specs)
    count, out_len = b.count, b.out_len
    m_tot, e_tot = int(b.m.sum()), int(len(b.col_idx))
    log(f"batch: {count} graphs, n={out_len} m={m_tot} generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(b.row_ptr).to(dev)
    ci = torch.from_numpy(b.col_idx).to(dev)
    tab, _ = dsg.batch_table(b.n, b.m, b.rp_off, b.ci_off, b.out_off, (num, den))
    torch.cuda.synchronize()

    if args.batch_shape:
        blk, it, bpc = (int(x) for x in args.batch_shape.split(","))
        shape, timings = {"block": blk, "walk_items": it, "blocks_per_cu": bpc}, []
    else:
        shape, timings = autotune.tune_batch(tab, count, len(b.row_ptr), e_tot, out_len, rp, ci,
                                             log=log)
    log(f"batch: autotuned shape {shape}")
    plan = dsg.Batch(tab, count, len(b.row_ptr), e_tot, out_len, launch=shape)
    best = torch.empty(max(out_len, 1), dtype=torch.int32, device=dev)
    res = torch.empty((count, dsg.RESULT_WORDS), dtype=torch.int64, device=dev)
    for _ in range(max(args.warmup, 1)):
        plan.run(rp, ci, best_ids=best, results=res)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.batch_steps):
        plan.run(rp, ci, best_ids=best, results=res)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t_start) * 1e3 / args.batch_steps
    # kernel time of the persistent launch alone, with events on the stream
    ev = []
    for _ in range(args.batch_steps):
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record()
        plan.run(rp, ci, best_ids=best, results=res)
        z.record()
        ev.append((a, z))
    torch.cuda.synchronize()
    ms_kernel = statistics.median(a.elapsed_time(z) for a, z in ev)
    got = dsg.Batch.results(res)
    bad = [i for i, r in enumerate(got) if r["status"] != 0]

    # one graph per call: the single-graph path on views of the same arrays
    ws = dsg.alloc_workspace(int(b.n.max()), int(b.m.max()), dev)
    one_best = torch.empty_like(best)
    order = range(count)
    torch.cuda.synchronize()
    t_one = time.perf_counter()
    for i in order:
        n_i, a_i, c_i, o_i = int(b.n[i]), int(b.rp_off[i]), int(b.ci_off[i]), int(b.out_off[i])
        dsg.peel(rp[a_i:a_i + n_i + 1], ci[c_i:c_i + 2 * int(b.m[i])], (num, den),
                 m=int(b.m[i]), best_ids=one_best[o_i:o_i + max(n_i, 1)], workspace=ws)
    torch.cuda.synchronize()
    s_one = time.perf_counter() - t_one
    one_gps = count / s_one
    gps = count / (ms_batch * 1e-3)
    # one pass over the CSR: every row is read once (4 B per entry), the
    # row offsets twice, the removal pass written once and read once
    alg_bytes = 4 * e_tot + 16 * out_len
    ach = alg_bytes / (ms_kernel * 1e-3) / 1e9
    log(f"batch: {ms_batch:.3f} ms per batch ({ms_kernel:.3f} ms kernel), {gps:,.0f} graphs/s; "
        f"one graph per call: {s_one:.2f} s, {one_gps:,.0f} graphs/s; x{gps / one_gps:.1f}")

    parity = None
    cpu = None
    if run_oracle:
        import oracle
        h_best = best.cpu().numpy()
        sample = list(range(0, count, max(count // 256, 1)))
        c0 = time.perf_counter()
        e_sample = 0
        same = not bad
        for i in sample:
            o = oracle.peel_graph(b.graph(i), num, den, trace=False)
            e_sample += int(b.m[i])
            r, a_i = got[i], int(b.out_off[i])
            same = same and (r["passes"], r["best_pass"], r["num"], r["den"]) == (
                o.passes, o.best_pass, o.num, o.den)
            same = same and bool((h_best[a_i:a_i + len(o.best)] == o.best).all())
        t_cpu = time.perf_counter() - c0
        # parity over every graph of the batch (the oracle on a thread pool:
        # each call is one C function that releases the interpreter lock)
        from concurrent.futures import ThreadPoolExecutor

        def one(i):
            o = oracle.peel_graph(b.graph(i), num, den, trace=False)
            r, a_i = got[i], int(b.out_off[i])
            return ((r["passes"], r["best_pass"], r["num"], r["den"]) == (
                o.passes, o.best_pass, o.num, o.den)
                and bool((h_best[a_i:a_i + len(o.best)] == o.best).all()))

        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as pool:
            same = same and all(pool.map(one, range(count)))
        parity = "exact" if same else "MISMATCH"
        cpu = dict({"value": round(len(sample) / t_cpu, 1), "unit": "graphs/s", "cores": 1,
                    "kind": "oracle",
                    "sample": f"{len(sample)} graphs (every {count // len(sample)}th, "
                              f"{e_sample} edges), single-threaded C oracle, {t_cpu:.2f} s"},
                   **host_cpu())
        log(f"batch oracle: sample of {len(sample)} graphs in {t_cpu:.2f} s on one core; "
            f"parity over all {count} graphs {parity}")
    return {
        "workload": (f"{count} graphs, n log-uniform [100, 100000], alternating Erdos-Renyi / "
                     f"Chung-Lu (gamma U[2.1, 2.8]), avg degree U[4, 64], seed 0, "
                     f"eps={num}/{den}"),
        "n": out_len, "m": m_tot,
        "graphs_per_s": round(gps, 1), "unit": "graphs/s",
        "ms_per_batch": round(ms_batch, 4), "ms_kernel": round(ms_kernel, 4),
        "one_graph_per_launch_graphs_per_s": round(one_gps, 1),
        "speedup_vs_one_graph_per_launch": round(gps / one_gps, 2),
        "gteps": round(m_tot / (ms_batch * 1e-3) / 1e9, 3),
        "shape": plan.shape,
        "autotune_candidates": len(timings),
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "kernel": "k_batch_peel", "alg_bytes_per_launch": alg_bytes},
        "status_errors": len(bad),
        "cpu_baseline": cpu,
        "parity": parity,
        "parity_scope": f"all {count} graphs" if parity else None,
    }



def bench_serve(args, torch) -> dict:
    """Latency and throughput of the serving loop under Poisson request
    streams at rising offered rates (the load curve).  Requests not admitted
    within 50 ms of arrival are shed, so the served rate saturates instead of
    collapsing and the served requests keep a bounded latency; the first
    (lowest) rate is also run without shedding.  Every served result is
    checked against the same graph and eps peeled alone by the single-graph
    path."""
    from paper_2103_00154_amd import dsg, inputs, serve
    eps_choices = ((1, 100), (1, 10), (1, 2))
    t0 = time.time()
    specs = inputs.serving_specs(args.serve_pool, seed=0)
    b = inputs.make_batch(specs)
    graphs = [b.graph(i) for i in range(b.count)]
    hg = [serve.HostGraph.from_graph(g) for g in graphs]
    log(f"serve: pool of {len(graphs)} graphs (n median {int(np.median(b.n))}, max "
        f"{int(b.n.max())}; m total {int(b.m.sum())}) built in {time.time() - t0:.1f}s")
    budget = 16 << 30
    shed_s = 0.05
    rates = [float(q) for q in args.serve_qps.split(",")]
    # warm-up: a short stream, not timed
    srv = serve.Server(budget, streams=args.serve_streams, max_batch=256)
    serve.run_load(srv, hg, eps_choices, qps=rates[0], count=64, seed=99)
    del srv
    curve, seen, same = [], {}, True
    runs = [(rates[0], None)] + [(q, shed_s) for q in rates]
    for qps, shed in runs:
        srv = serve.Server(budget, streams=args.serve_streams, max_batch=256, max_queue_s=shed)
        reqs = serve.run_load(srv, hg, eps_choices, qps=qps, count=args.serve_requests, seed=7)
        torch.cuda.synchronize()
        st = serve.latency_stats(reqs)
        point = dict(st, offered_qps=qps, shed_after_ms=None if shed is None else shed * 1e3,
                     micro_batches=srv.batches,
                     mean_batch=round(float(np.mean(srv.batch_sizes)), 2) if srv.batch_sizes
                     else 0.0,
                     lane_requests=srv.big_done, arena_peak_bytes=srv.arena.peak)
        curve.append(point)
        big_vertices = srv.big_vertices
        log(f"serve {qps:g} req/s (shed {'off' if shed is None else f'{shed * 1e3:g} ms'}): "
            f"{st}; {srv.batches} micro-batches, {srv.big_done} large requests in the lane")
        same = same and all(r.result["status"] == 0 for r in reqs if not r.rejected)
        for r in reqs:
            if not r.rejected:
                seen.setdefault((r.rid % len(graphs), r.eps), []).append(r)
    # every (graph, eps) pair that was served, peeled alone
    for (gi, e), rs in seen.items():
        g = graphs[gi]
        rp = torch.from_numpy(g.row_ptr).cuda()
        ci = torch.from_numpy(g.col_idx if g.m else np.zeros(1, np.int32)).cuda()
        a = dsg.peel(rp, ci, e, m=g.m)
        ab = a.best.cpu().numpy()
        for r in rs:
            same = same and (r.result["num"], r.result["den"], r.result["passes"],
                             r.result["best_pass"]) == (a.num, a.den, a.passes, a.best_pass)
            same = same and np.array_equal(r.best, ab)
    parity = "exact" if same else "MISMATCH"
    log(f"serve: results vs peeled alone: {parity} ({len(seen)} graph/eps pairs)")
    head = curve[0]
    return dict(head, **{
        "workload": (f"Poisson streams of Chung-Lu graphs, n lognormal (median 20000, sigma 1, "
                     f"capped at 2000000), avg degree U[8, 64], gamma U[2.1, 2.8], eps from "
                     f"{{1/100, 1/10, 1/2}}; pool of {len(graphs)} graphs, each request uploads "
                     f"its CSR; {args.serve_requests} requests per offered rate"),
        "budget_bytes": budget, "streams": args.serve_streams,
        "large_request_lane": {"above_vertices": big_vertices, "entry": "dsg_peel_async"},
        "load_curve": curve,
        "parity": parity})


def bench_sweep(args, torch, run_oracle: bool) -> dict:
    """The peel of R-MAT scale 20 at eps from 0 to 5: passes, density, time
    per eps and rho(S~) / rho* against the exact densest subgraph computed on
    the GPU, each against the oracle (parity and the oracle's time)."""
    from paper_2103_00154_amd import dsg, inputs, sweep
    eps_list = ((0, 1), (1, 100), (1, 20), (1, 10), (1, 2), (1, 1), (2, 1), (5, 1))
    g = inputs.rmat(20, 16, seed=0)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    pts = sweep.eps_sweep(rp, ci, eps_list, reps=5)
    x0 = time.perf_counter()
    x = dsg.exact_density(rp, ci, extract=False)
    x_s = time.perf_counter() - x0
    log(f"sweep: exact rho* = {x.num}/{x.den} on the GPU in {x_s:.2f} s ({x.flows} flows, "
        f"{x.relabels} global relabels)")
    for pt in pts:
        pt.ratio = pt.num * x.den / (pt.den * x.num)
    rows = []
    same = True
    for pt in pts:
        row = {"eps": f"{pt.eps[0]}/{pt.eps[1]}", "passes": pt.passes, "best_pass": pt.best_pass,
               "dens_num": pt.num, "dens_den": pt.den, "density": round(pt.density, 3),
               "ms": round(pt.ms, 4), "gteps": round(g.m / (pt.ms * 1e-3) / 1e9, 2),
               "removed_per_pass": [t["removed"] for t in pt.trace],
               "ratio_to_exact": round(pt.ratio, 6)}
        if run_oracle:
            import oracle
            c0 = time.perf_counter()
            o = oracle.peel_graph(g, *pt.eps, trace=True)
            row["oracle_ms"] = round((time.perf_counter() - c0) * 1e3, 1)
            ok = (pt.passes, pt.best_pass, pt.num, pt.den) == (o.passes, o.best_pass, o.num,
                                                                o.den)
            ok = ok and [t["removed"] for t in pt.trace] == [t["removed"] for t in o.trace]
            same = same and ok
        rows.append(row)
        log(f"sweep eps {row['eps']}: passes {pt.passes}, best {pt.num}/{pt.den}, "
            f"rho(S~)/rho* {pt.ratio:.4f}, {pt.ms:.3f} ms")
    return {"workload": "R-MAT scale 20, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed 0",
            "n": g.n, "m": g.m, "points": rows,
            "exact_density": [x.num, x.den], "exact_flows": x.flows, "exact_s": round(x_s, 3),
            "parity": ("exact" if same else "MISMATCH") if run_oracle else None,
            "cpu_baseline_kind": "oracle" if run_oracle else None}


def bench_cbds(args, torch, run_oracle: bool) -> dict:
    """CBDS-P (Section 3.2, Algorithm 2) on R-MAT scale 20 and on the
    scale-24 workload: device time, levels and passes, the densest core and
    the extension, next to the peel's densities at eps = 0 and 1/10 (the
    comparison the paper's Table 3 makes); parity and time of the oracle."""
    import statistics as stt
    from paper_2103_00154_amd import dsg, inputs
    runs = []
    for name in ("rmat20", "rmat24"):
        g = inputs.rmat(20, 16, seed=0) if name == "rmat20" else \
            inputs.rmat(24, 16, seed=0, planted=(2000, 0.5, 1))
        rp = torch.from_numpy(g.row_ptr).cuda()
        ci = torch.from_numpy(g.col_idx).cuda()
        ws = dsg.alloc_workspace(g.n, g.m)
        r = dsg.cbds(rp, ci, workspace=ws)
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = dsg.cbds(rp, ci, workspace=ws)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        ms = stt.median(times)
        p0 = dsg.peel(rp, ci, (0, 1), workspace=ws)
        p1 = dsg.peel(rp, ci, (1, 10), workspace=ws)
        row = {"workload": name, "n": g.n, "m": g.m, "ms": round(ms, 3),
               "gteps": round(g.m / (ms * 1e-3) / 1e9, 3), "passes": r.passes, "kmax": r.kmax,
               "core_k": r.K, "core_density": [r.core_num, r.core_den],
               "eligible": r.n_eligible, "legit": r.n_legit, "density": [r.num, r.den],
               "density_value": round(r.num / r.den, 3),
               "peel_eps0_density": [p0.num, p0.den], "peel_eps_1_10_density": [p1.num, p1.den]}
        if run_oracle:
            import oracle
            c0 = time.perf_counter()
            o = oracle.cbds(g)
            row["oracle_ms"] = round((time.perf_counter() - c0) * 1e3, 1)
            same = (r.num, r.den, r.core_num, r.core_den, r.K, r.n_legit, r.kmax) == (
                o.num, o.den, o.core_num, o.core_den, o.K, o.n_legit, o.kmax)
            same = same and np.array_equal(r.best.cpu().numpy(), o.best)
            row["parity"] = "exact" if same else "MISMATCH"
        else:
            row["parity"] = None
        log(f"cbds {name}: {ms:.3f} ms ({row['gteps']} GTEPS), {r.passes} passes, kmax {r.kmax}, "
            f"K {r.K}, legit {r.n_legit}, density {r.num}/{r.den} = {r.num / r.den:.3f} "
            f"(peel eps=0: {p0.num}/{p0.den} = {p0.num / p0.den:.3f}); parity {row['parity']}")
        runs.append(row)
        del rp, ci, ws
    return {"runs": runs}


if __name__ == "__main__":
    sys.exit(main())
