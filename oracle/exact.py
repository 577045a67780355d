"""Exact densest-subgraph densities, used to check the (2+2eps) guarantee.

TEST INFRASTRUCTURE.  Two independent routes:

* :func:`densest_bruteforce` - max over every non-empty vertex subset of
  |E(S)| / |S| (Definition 1); feasible for n <= ~16.
* :func:`densest_goldberg`   - Goldberg's max-flow construction (cited in
  Section 2 as the exact method) inside a Dinkelbach iteration.  For a guess
  g = p/q the network has s->v with capacity q*m, v->t with capacity
  q*m + 2p - q*deg(v), and capacity q on both arcs of every edge; a cut with
  source side {s} + S costs q*m*n + 2(p|S| - q|E(S)|), so some S beats g
  exactly when the minimum cut is below q*m*n.  scipy's max-flow is the
  flow primitive.
* :func:`densest_maximal`    - the largest densest subgraph (the union of all
  subsets of greatest density) from the largest minimum-cut side of the same
  network with its constant terms dropped (capacities small enough for the
  int32 flow primitive at 10^5 vertices); pinned against brute force and
  against :func:`densest_goldberg`.
"""
from __future__ import annotations

from fractions import Fraction
from math import gcd

import numpy as np


def densest_bruteforce(n: int, edges) -> tuple[int, int, list[int]]:
    """(|E(S*)|, |S*|, S*) maximising |E(S)|/|S|; among equal densities the
    first subset in bitmask order wins."""
    if n == 0:
        return 0, 0, []
    adj = [0] * n
    for u, v in edges:
        adj[u] |= 1 << v
        adj[v] |= 1 << u
    best = (0, 1, 1)  # (E, |S|, mask) of the singleton {0}
    for mask in range(1, 1 << n):
        size = bin(mask).count("1")
        twice_e = 0
        rest = mask
        while rest:
            low = rest & -rest
            v = low.bit_length() - 1
            twice_e += bin(adj[v] & mask).count("1")
            rest ^= low
        e = twice_e // 2
        if e * best[1] > best[0] * size:
            best = (e, size, mask)
    e, s, mask = best
    return e, s, [v for v in range(n) if mask >> v & 1]


def _induced(edge_arr: np.ndarray, members: np.ndarray) -> int:
    if len(edge_arr) == 0:
        return 0
    return int(np.count_nonzero(members[edge_arr[:, 0]] & members[edge_arr[:, 1]]))


def _min_cut_side(n, edge_arr, deg, m, p, q):
    """Source side (without s) of a minimum s-t cut, and the cut value."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_flow, breadth_first_order

    s, t = n, n + 1
    rows = [np.full(n, s), np.arange(n), edge_arr[:, 0], edge_arr[:, 1]]
    cols = [np.arange(n), np.full(n, t), edge_arr[:, 1], edge_arr[:, 0]]
    caps = [np.full(n, q * m), q * m + 2 * p - q * deg, np.full(len(edge_arr), q),
            np.full(len(edge_arr), q)]
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    w = np.concatenate(caps).astype(np.int64)
    if w.max(initial=0) >= 2**31 or w.min(initial=0) < 0:
        raise OverflowError("capacities outside the int32 range of the flow primitive")
    cap = csr_matrix((w.astype(np.int32), (r, c)), shape=(n + 2, n + 2))
    res = maximum_flow(cap, s, t)
    flow = res.flow.tocsr()
    resid = (cap.astype(np.int64) - flow.astype(np.int64)).tocsr()
    resid.data[resid.data < 0] = 0
    resid.eliminate_zeros()
    reach = breadth_first_order(resid, s, directed=True, return_predecessors=False)
    side = np.zeros(n + 2, dtype=bool)
    side[reach] = True
    return side[:n], int(res.flow_value)


def densest_goldberg(n: int, edges) -> tuple[int, int, np.ndarray]:
    """(|E(S*)|, |S*|, S* as bool mask) via Goldberg cuts + Dinkelbach."""
    edge_arr = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    m = len(edge_arr)
    if n == 0:
        return 0, 0, np.zeros(0, dtype=bool)
    if m == 0:
        mask = np.zeros(n, dtype=bool)
        mask[0] = True
        return 0, 1, mask
    deg = np.bincount(edge_arr.ravel(), minlength=n).astype(np.int64)
    members = np.ones(n, dtype=bool)
    e_cur, s_cur = m, n
    while True:
        g = gcd(e_cur, s_cur)
        p, q = e_cur // g, s_cur // g
        side, cut = _min_cut_side(n, edge_arr, deg, m, p, q)
        if cut >= q * m * n:
            return e_cur, s_cur, members
        e_new, s_new = _induced(edge_arr, side), int(side.sum())
        if s_new == 0 or Fraction(e_new, s_new) <= Fraction(e_cur, s_cur):
            raise AssertionError("Goldberg cut did not improve the density")
        e_cur, s_cur, members = e_new, s_new, side


def _maximal_min_cut_side(n, edge_arr, deg, p, q):
    """Largest source side (without s) among the minimum cuts of Goldberg's
    network for the guess p/q, written without its constant terms: s->v with
    capacity max(0, q*deg(v) - 2p), v->t with capacity max(0, 2p - q*deg(v))
    and capacity q on both arcs of every edge.  A cut with source side
    {s} + S then costs cut({s}) + 2(p|S| - q|E(S)|): the minimum cuts are
    Goldberg's, with capacities of at most max(q*deg, 2p).  The largest
    source side is the set of vertices from which t cannot be reached in the
    residual graph of a maximum flow."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_flow, breadth_first_order

    s, t = n, n + 1
    a = q * deg - 2 * p
    src = np.flatnonzero(a > 0)
    snk = np.flatnonzero(a < 0)
    rows = [np.full(len(src), s), snk, edge_arr[:, 0], edge_arr[:, 1]]
    cols = [src, np.full(len(snk), t), edge_arr[:, 1], edge_arr[:, 0]]
    caps = [a[src], -a[snk], np.full(len(edge_arr), q), np.full(len(edge_arr), q)]
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    w = np.concatenate(caps).astype(np.int64)
    if w.max(initial=0) >= 2**31:
        raise OverflowError("capacities outside the int32 range of the flow primitive")
    cap = csr_matrix((w.astype(np.int32), (r, c)), shape=(n + 2, n + 2))
    flow = maximum_flow(cap, s, t).flow.tocsr()
    resid = (cap.astype(np.int64) - flow.astype(np.int64)).tocsr()
    resid.data[resid.data < 0] = 0
    resid.eliminate_zeros()
    # vertices that reach t: search from t along reversed residual arcs
    reach = breadth_first_order(resid.transpose().tocsr(), t, directed=True,
                                return_predecessors=False)
    side = np.ones(n + 2, dtype=bool)
    side[reach] = False
    return side[:n]


def densest_maximal(n: int, edges) -> tuple[int, int, np.ndarray]:
    """(|E(S*)|, |S*|, S* as bool mask) for the largest densest subgraph S*
    (the union of all subsets of greatest density, itself of that density),
    by Dinkelbach's iteration over the largest minimum-cut side of
    Goldberg's network: starting from the density of G, each cut side that
    is strictly denser becomes the next guess; the side at the optimum
    guess is S*.  The edgeless graph gives S* = V with density 0."""
    edge_arr = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    m = len(edge_arr)
    if n == 0:
        return 0, 0, np.zeros(0, dtype=bool)
    deg = np.bincount(edge_arr.ravel(), minlength=n).astype(np.int64)
    e_cur, s_cur = m, n
    while True:
        g = gcd(e_cur, s_cur)
        p, q = e_cur // g, s_cur // g
        side = _maximal_min_cut_side(n, edge_arr, deg, p, q)
        e_new, s_new = _induced(edge_arr, side), int(side.sum())
        if s_new > 0 and e_new * s_cur > e_cur * s_new:
            e_cur, s_cur = e_new, s_new
            continue
        if s_new == 0 or e_new * s_cur != e_cur * s_new:
            raise AssertionError("the cut side at the optimum guess is not of that density")
        return e_new, s_new, side
