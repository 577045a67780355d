"""CBDS-P (Section 3.2, Algorithm 2) restated from definitions, for small
graphs.  TEST INFRASTRUCTURE ONLY.

* The k-core is the largest subgraph in which every vertex has degree >= k
  (Section 2): it is what is left after deleting vertices of degree < k until
  none is left.  The core number of v is the largest k whose k-core holds v.
* The densest core is the non-empty k-core of greatest |E|/|V| (smallest k
  among equal densities).
* With rho its density, an outside vertex v joins when its core number
  exceeds rho (eligible) and its number of neighbours inside the core exceeds
  rho (legitimate).  All such vertices join together.

Every count is recomputed from the edge list; densities are Fractions.
``printed_label=True`` records the order of the core as the level k that was
peeled just before it (k - 1 here), as the printed algorithm does; the
comparison tests use it to show why that reading is not taken.
"""
from __future__ import annotations

from fractions import Fraction


def _adj(n, edges):
    adj = [set() for _ in range(n)]
    for u, v in edges:
        adj[u].add(v)
        adj[v].add(u)
    return adj


def k_core(n, adj, k) -> set:
    alive = set(range(n))
    changed = True
    while changed:
        changed = False
        for v in list(alive):
            if len(adj[v] & alive) < k:
                alive.discard(v)
                changed = True
    return alive


def induced_edges(adj, members) -> int:
    return sum(len(adj[v] & members) for v in members) // 2


def cbds_literal(n: int, edges, printed_label: bool = False) -> dict:
    adj = _adj(n, edges)
    if n == 0:
        return {"num": 0, "den": 0, "K": 0, "core": [], "legit": [], "best": [],
                "claimed": (0, 0)}
    maxdeg = max(len(a) for a in adj)
    cores = [k_core(n, adj, k) for k in range(maxdeg + 2)]
    core = [max(k for k in range(maxdeg + 1) if v in cores[k]) for v in range(n)]
    best_k, best_d = 0, None
    for k, c in enumerate(cores):
        if not c:
            break
        d = Fraction(induced_edges(adj, c), len(c))
        if best_d is None or d > best_d:
            best_k, best_d = k, d
    K = best_k - 1 if printed_label and best_k > 0 else best_k
    inner = {v for v in range(n) if core[v] >= K}   # the set the label selects
    me, mv = induced_edges(adj, cores[best_k]), len(cores[best_k])
    rho = Fraction(me, mv)
    legit = []
    sum_legits = 0
    for v in range(n):
        if core[v] >= K or not core[v] > rho:
            continue
        legits = len(adj[v] & inner)
        if legits > rho:
            legit.append(v)
            sum_legits += legits
    e_l = induced_edges(adj, set(legit))
    members = inner | set(legit)
    return {"num": induced_edges(adj, members), "den": len(members), "K": K, "core": core,
            "legit": legit, "best": sorted(members),
            # the density the algorithm reports: core counts plus the additions
            "claimed": (me + sum_legits + e_l, mv + len(legit)),
            "core_num": me, "core_den": mv}
