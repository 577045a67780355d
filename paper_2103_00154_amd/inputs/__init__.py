"""Seeded synthetic inputs: undirected simple graphs as int32 CSR.

This module is shared by the CPU oracle's tests and by the GPU library's
tests and benchmark.  It builds inputs only and holds none of the peeling
arithmetic.  Big generators run in ``libgraphgen.so`` (host C, OpenMP,
counter-based randomness, so results do not depend on the thread count);
tiny fixed graphs are built with numpy by :func:`from_edges`.

Every CSR produced here is symmetric, has no self loops or repeated edges,
and lists each row's neighbours in ascending order.  ``m`` counts undirected
edges, so ``len(col_idx) == 2 * m``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Iterable, Sequence

import numpy as np

from .. import _build

_U64 = ctypes.c_uint64
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_P = ctypes.c_void_p

_lib = None


def _gen():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(str(_build.ensure_graphgen()))
        lib.gg_rmat_keys.argtypes = [_I32, _I64, _U64, _U64, _U64, _U64, _U64, _P]
        lib.gg_rmat_keys.restype = _I64
        lib.gg_er_keys.argtypes = [_I64, _I64, _U64, _U64, _P]
        lib.gg_er_keys.restype = _I64
        lib.gg_planted_keys.argtypes = [_I64, _I64, _U64, _U64, _U64, _P, _P]
        lib.gg_planted_keys.restype = _I64
        lib.gg_chung_lu_keys.argtypes = [_I64, _I64, ctypes.c_double, _U64, _U64, _P]
        lib.gg_chung_lu_keys.restype = _I64
        lib.gg_sort_unique.argtypes = [_P, _P, _I64]
        lib.gg_sort_unique.restype = _I64
        lib.gg_keys_to_csr.argtypes = [_P, _I64, _I64, _P, _P]
        lib.gg_keys_to_csr.restype = _I32
        lib.gg_draw_for_test.argtypes = [_U64, _U64, _U64]
        lib.gg_draw_for_test.restype = _U64
        lib.gg_batch_generate.argtypes = [_I32, _P, _P, _P, _P, _P, _P]
        lib.gg_batch_generate.restype = _P
        lib.gg_batch_copy.argtypes = [_P, _P, _P, _P, _P]
        lib.gg_batch_copy.restype = _I32
        lib.gg_batch_free.argtypes = [_P]
        lib.gg_batch_free.restype = None
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Undirected simple graph on vertices 0..n-1 in CSR form."""

    n: int
    m: int
    row_ptr: np.ndarray  # int32[n + 1]
    col_idx: np.ndarray  # int32[2m]
    name: str = ""
    meta: dict = field(default_factory=dict)

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def edges(self) -> np.ndarray:
        """Undirected edges (u < v) as an int64 array of shape (m, 2)."""
        deg = self.degrees()
        src = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        dst = self.col_idx.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _keys_to_graph(keys: np.ndarray, count: int, n: int, name: str, meta: dict) -> Graph:
    lib = _gen()
    tmp = np.empty(max(count, 1), dtype=np.uint64)
    uniq = lib.gg_sort_unique(_ptr(keys), _ptr(tmp), count)
    del tmp
    if uniq < 0:
        raise MemoryError("gg_sort_unique failed")
    if uniq > 0x7FFFFFFF:
        raise OverflowError(f"{uniq} adjacency entries exceed the int32 CSR range")
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col_idx = np.empty(max(uniq, 1), dtype=np.int32)
    rc = lib.gg_keys_to_csr(_ptr(keys), uniq, n, _ptr(row_ptr), _ptr(col_idx))
    if rc != 0:
        raise ValueError("edge keys do not fit the vertex range")
    col_idx = col_idx[:uniq].copy() if uniq else np.empty(0, dtype=np.int32)
    assert uniq % 2 == 0
    return Graph(n=n, m=uniq // 2, row_ptr=row_ptr, col_idx=col_idx, name=name, meta=meta)


# --------------------------------------------------------------------------
# generators
# --------------------------------------------------------------------------

def erdos_renyi(n: int, m: int, seed: int = 0) -> Graph:
    """G(n, m): uniform vertex pairs, loops and repeated edges rejected until
    exactly m distinct edges exist."""
    if n < 0 or m < 0 or 2 * m > n * max(n - 1, 0):
        raise ValueError(f"G({n}, {m}) does not exist")
    keys = np.empty(max(2 * m, 1), dtype=np.uint64)
    cnt = _gen().gg_er_keys(n, m, seed, 1, _ptr(keys))
    if cnt < 0:
        raise ValueError("gg_er_keys rejected its arguments")
    return _keys_to_graph(keys, cnt, n, f"er_n{n}_m{m}_s{seed}",
                          {"kind": "er", "seed": seed})


def _fix32(x: float) -> int:
    return min(int(x * 2**32), 2**32)


def rmat(scale: int, edge_factor: int = 16, abcd: Sequence[float] = (0.57, 0.19, 0.19, 0.05),
         seed: int = 0, planted: tuple[int, float, int] | None = None) -> Graph:
    """R-MAT graph with 2^scale vertices and edge_factor * 2^scale samples;
    loops and repeats are dropped, so m is the realised edge count.

    ``planted=(k, p, seed)`` adds G(k, p) on k distinct random vertex ids;
    the chosen ids are returned in ``meta['planted_ids']``.
    """
    a, b, c, d = abcd
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("R-MAT probabilities must sum to 1")
    n = 1 << scale
    ns = edge_factor * n
    extra = 0
    if planted is not None:
        k = planted[0]
        extra = k * (k - 1)
    keys = np.empty(2 * ns + extra, dtype=np.uint64)
    lib = _gen()
    cnt = lib.gg_rmat_keys(scale, ns, _fix32(a), _fix32(a + b), _fix32(a + b + c), seed, 2,
                           _ptr(keys))
    if cnt < 0:
        raise ValueError("gg_rmat_keys rejected its arguments")
    meta = {"kind": "rmat", "scale": scale, "edge_factor": edge_factor, "abcd": tuple(abcd),
            "seed": seed}
    name = f"rmat_s{scale}_ef{edge_factor}_s{seed}"
    if planted is not None:
        k, p, pseed = planted
        ids = np.empty(max(k, 1), dtype=np.int32)
        p_fix = min(int(p * 2**64), 2**64 - 1)
        got = lib.gg_planted_keys(n, k, p_fix, pseed, 3, _ptr(ids), _ptr(keys[cnt:]))
        if got < 0:
            raise ValueError("gg_planted_keys rejected its arguments")
        cnt += got
        meta["planted_ids"] = ids[:k].copy()
        meta["planted"] = (k, p, pseed)
        name += f"_planted{k}"
    return _keys_to_graph(keys, cnt, n, name, meta)


def chung_lu(n: int, avg_deg: float, gamma: float, seed: int = 0) -> Graph:
    """Chung-Lu power-law graph: weights (i+1)^(-1/(gamma-1)); round(n*avg_deg/2)
    endpoint pairs drawn proportionally to weight; loops and repeats dropped."""
    npairs = int(round(n * avg_deg / 2))
    keys = np.empty(max(2 * npairs, 1), dtype=np.uint64)
    cnt = _gen().gg_chung_lu_keys(n, npairs, float(gamma), seed, 4, _ptr(keys))
    if cnt < 0:
        raise ValueError("gg_chung_lu_keys rejected its arguments")
    return _keys_to_graph(keys, cnt, n, f"cl_n{n}_d{avg_deg}_g{gamma}_s{seed}",
                          {"kind": "chung_lu", "gamma": gamma, "avg_deg": avg_deg, "seed": seed})


# --------------------------------------------------------------------------
# small fixed graphs (numpy only)
# --------------------------------------------------------------------------

def from_edges(n: int, edges: Iterable[Sequence[int]], name: str = "") -> Graph:
    """CSR of the simple undirected graph with the given edge set.  Loops are
    rejected; repeated edges collapse to one."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if e.size and (e.min() < 0 or e.max() >= n):
        raise ValueError("edge endpoint outside 0..n-1")
    if np.any(e[:, 0] == e[:, 1]):
        raise ValueError("self loops are not part of the input domain")
    both = np.concatenate([e, e[:, ::-1]], axis=0)
    keys = np.unique(both[:, 0] * (n + 1) + both[:, 1]) if both.size else np.empty(0, np.int64)
    src = keys // (n + 1)
    dst = keys % (n + 1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return Graph(n=n, m=len(keys) // 2, row_ptr=row_ptr, col_idx=dst.astype(np.int32),
                 name=name or f"edges_n{n}")


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Graph with vertex v renamed perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    e = g.edges()
    return from_edges(g.n, perm[e] if len(e) else e, name=g.name + "_relabel")


def clique(k: int, offset: int = 0, n: int | None = None) -> Graph:
    n = k + offset if n is None else n
    return from_edges(n, [(offset + i, offset + j) for i in range(k) for j in range(i + 1, k)],
                      name=f"K{k}")


def star(n: int) -> Graph:
    return from_edges(n, [(0, i) for i in range(1, n)], name=f"star{n}")


def path(n: int) -> Graph:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], name=f"path{n}")


def cycle(n: int) -> Graph:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)] if n >= 3 else [], name=f"C{n}")


def empty(n: int) -> Graph:
    return from_edges(n, [], name=f"empty{n}")


def disjoint_cliques(a: int, b: int) -> Graph:
    edges = [(i, j) for i in range(a) for j in range(i + 1, a)]
    edges += [(a + i, a + j) for i in range(b) for j in range(i + 1, b)]
    return from_edges(a + b, edges, name=f"K{a}+K{b}")


def random_small(n: int, p: float, seed: int) -> Graph:
    """G(n, p) for tiny test graphs (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return from_edges(n, edges, name=f"gnp_n{n}_p{p}_s{seed}")


def draw_for_test(seed: int, stream: int, i: int) -> int:
    return int(_gen().gg_draw_for_test(seed, stream, i))


# --------------------------------------------------------------------------
# batches of independent graphs, stored back to back
# --------------------------------------------------------------------------

KIND_ER = 0
KIND_CHUNG_LU = 1


@dataclass
class GraphSpec:
    """Recipe of one batch graph: G(n, size) for kind 0, Chung-Lu with
    ``size`` endpoint pairs and exponent ``gamma`` for kind 1."""

    kind: int
    n: int
    size: int
    gamma: float
    seed: int
    avg_deg: float


@dataclass
class Batch:
    """Graphs stored back to back: graph i has n[i] vertices and m[i] edges,
    its local row offsets at row_ptr[rp_off[i] : rp_off[i] + n[i] + 1], its
    neighbour ids at col_idx[ci_off[i] : ci_off[i] + 2 m[i]], and owns the
    output slots out_off[i] : out_off[i] + n[i]."""

    n: np.ndarray        # int64[count]
    m: np.ndarray        # int64[count]
    rp_off: np.ndarray   # int64[count]
    ci_off: np.ndarray   # int64[count]
    out_off: np.ndarray  # int64[count]
    row_ptr: np.ndarray  # int32[sum(n + 1)]
    col_idx: np.ndarray  # int32[sum(2 m)]
    specs: list

    @property
    def count(self) -> int:
        return len(self.n)

    @property
    def out_len(self) -> int:
        return int(self.n.sum())

    def graph(self, i: int) -> Graph:
        n, a, b = int(self.n[i]), int(self.rp_off[i]), int(self.ci_off[i])
        m = int(self.m[i])
        sp = self.specs[i]
        meta = {"kind": sp.kind, "seed": sp.seed} if sp is not None else {}
        return Graph(n=n, m=m, row_ptr=self.row_ptr[a:a + n + 1].copy(),
                     col_idx=self.col_idx[b:b + 2 * m].copy(), name=f"batch_{i}", meta=meta)


def batch_specs(count: int, seed: int = 0, n_range=(100, 100_000), deg_range=(4.0, 64.0),
                gamma_range=(2.1, 2.8)) -> list[GraphSpec]:
    """Recipes for a mixed batch: n log-uniform in n_range, average degree
    uniform in deg_range, graphs alternating Erdos-Renyi and Chung-Lu with
    exponent uniform in gamma_range.  The parameters are drawn with numpy's
    PCG64 under ``seed``; graph i is generated under seed (seed << 32) + i."""
    rng = np.random.default_rng(seed)
    lo, hi = np.log(n_range[0]), np.log(n_range[1])
    specs = []
    for i in range(count):
        n = int(round(float(np.exp(rng.uniform(lo, hi)))))
        d = float(rng.uniform(*deg_range))
        g = float(rng.uniform(*gamma_range))
        gseed = (int(seed) << 32) + i
        if i % 2 == 0:
            m = min(int(round(n * d / 2)), n * (n - 1) // 2)
            specs.append(GraphSpec(KIND_ER, n, m, 0.0, gseed, d))
        else:
            specs.append(GraphSpec(KIND_CHUNG_LU, n, int(round(n * d / 2)), g, gseed, d))
    return specs


def serving_specs(count: int, seed: int = 0, median: float = 20_000, sigma: float = 1.0,
                  n_cap: int = 2_000_000, deg_range=(8.0, 64.0),
                  gamma_range=(2.1, 2.8)) -> list[GraphSpec]:
    """Recipes of request graphs: Chung-Lu with n lognormal (the given median
    and sigma, clipped to [100, n_cap]), average degree uniform in deg_range
    and exponent uniform in gamma_range; numpy PCG64 under ``seed``, graph i
    generated under seed (seed << 32) + (1 << 31) + i."""
    rng = np.random.default_rng(seed + 0x5E5)
    specs = []
    for i in range(count):
        n = int(min(max(round(float(rng.lognormal(np.log(median), sigma))), 100), n_cap))
        d = float(rng.uniform(*deg_range))
        g = float(rng.uniform(*gamma_range))
        specs.append(GraphSpec(KIND_CHUNG_LU, n, int(round(n * d / 2)), g,
                               (int(seed) << 32) + (1 << 31) + i, d))
    return specs


def make_batch(specs: Sequence[GraphSpec]) -> Batch:
    """Generate every graph of ``specs`` (in parallel, one graph per thread)
    and lay them out back to back."""
    count = len(specs)
    kind = np.array([s.kind for s in specs], dtype=np.int32)
    n = np.array([s.n for s in specs], dtype=np.int64)
    size = np.array([s.size for s in specs], dtype=np.int64)
    gamma = np.array([s.gamma for s in specs], dtype=np.float64)
    seeds = np.array([s.seed for s in specs], dtype=np.uint64)
    m = np.zeros(count, dtype=np.int64)
    lib = _gen()
    h = lib.gg_batch_generate(count, _ptr(kind), _ptr(n), _ptr(size), _ptr(gamma), _ptr(seeds),
                              _ptr(m))
    if not h:
        raise ValueError("gg_batch_generate failed (bad recipe or out of memory)")
    try:
        rp_off = np.zeros(count, dtype=np.int64)
        ci_off = np.zeros(count, dtype=np.int64)
        if count:
            rp_off[1:] = np.cumsum(n + 1)[:-1]
            ci_off[1:] = np.cumsum(2 * m)[:-1]
        out_off = rp_off - np.arange(count, dtype=np.int64)
        row_ptr = np.empty(max(int((n + 1).sum()), 1), dtype=np.int32)
        col_idx = np.empty(max(int((2 * m).sum()), 1), dtype=np.int32)
        if lib.gg_batch_copy(h, _ptr(row_ptr), _ptr(col_idx), _ptr(rp_off), _ptr(ci_off)) != 0:
            raise ValueError("gg_batch_copy failed")
    finally:
        lib.gg_batch_free(h)
    return Batch(n=n, m=m, rp_off=rp_off, ci_off=ci_off, out_off=out_off, row_ptr=row_ptr,
                 col_idx=col_idx, specs=list(specs))


def concat(graphs: Sequence[Graph]) -> Batch:
    """Lay out existing graphs back to back as a batch."""
    count = len(graphs)
    n = np.array([g.n for g in graphs], dtype=np.int64)
    m = np.array([g.m for g in graphs], dtype=np.int64)
    rp_off = np.zeros(count, dtype=np.int64)
    ci_off = np.zeros(count, dtype=np.int64)
    if count:
        rp_off[1:] = np.cumsum(n + 1)[:-1]
        ci_off[1:] = np.cumsum(2 * m)[:-1]
    out_off = rp_off - np.arange(count, dtype=np.int64)
    row_ptr = np.empty(max(int((n + 1).sum()), 1), dtype=np.int32)
    col_idx = np.empty(max(int((2 * m).sum()), 1), dtype=np.int32)
    for i, g in enumerate(graphs):
        row_ptr[rp_off[i]:rp_off[i] + g.n + 1] = g.row_ptr
        col_idx[ci_off[i]:ci_off[i] + 2 * g.m] = g.col_idx[:2 * g.m]
    return Batch(n=n, m=m, rp_off=rp_off, ci_off=ci_off, out_off=out_off, row_ptr=row_ptr,
                 col_idx=col_idx, specs=[None] * count)
