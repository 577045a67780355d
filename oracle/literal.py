"""Literal peeling oracle: Algorithm 1 (P-Bahmani, Section 3.1) with every
quantity recomputed from its definition in every pass.

TEST INFRASTRUCTURE (pure Python, tiny graphs).  Unlike the C oracle it keeps
no running degrees or edge counts: the degree of v is |N(v) & S| and |E(S)|
is counted over the edge list (Definition 1) each time they are needed.  It
is used to pin the C oracle on exhaustive and random small graphs.
"""
from __future__ import annotations


def _induced_edges(edges, S):
    return sum(1 for (u, v) in edges if u in S and v in S)


def peel_literal(n: int, edges, eps_num: int, eps_den: int) -> dict:
    """Return passes, best pass, (|E(S~)|, |S~|), S~ (sorted), removal pass
    of every vertex and a per-pass trace (same fields as the C oracle)."""
    edges = [(min(u, v), max(u, v)) for (u, v) in edges]
    adj = {v: set() for v in range(n)}
    for u, v in edges:
        adj[u].add(v)
        adj[v].add(u)
    S = set(range(n))
    removed_at = [None] * n
    best = (_induced_edges(edges, S), len(S), 0)
    trace = []
    k = 0
    while S:
        k += 1
        V = len(S)
        E = _induced_edges(edges, S)
        # part 1: deg_S(v) <= 2 (1 + eps) E / V, exactly in integers
        failed = {v for v in S if len(adj[v] & S) * V * eps_den <= 2 * (eps_num + eps_den) * E}
        for v in failed:
            removed_at[v] = k
        S_next = S - failed
        E_next = _induced_edges(edges, S_next)
        trace.append({
            "s_in": V, "e_in": E,
            "thresh": (2 * (eps_num + eps_den) * E) // (V * eps_den),
            "removed": len(failed),
            "cross": sum(len(adj[v] & S_next) for v in failed),
            "intra": sum(len(adj[v] & failed) for v in failed),
            "scanned": sum(len(adj[v]) for v in failed),
            "s_out": len(S_next), "e_out": E_next,
        })
        if S_next and E_next * best[1] > best[0] * len(S_next):
            best = (E_next, len(S_next), k)
        S = S_next
    best_set = sorted(v for v in range(n) if removed_at[v] > best[2])
    return {"passes": k, "best_pass": best[2], "num": best[0], "den": best[1],
            "best": best_set, "removed_at": removed_at, "trace": trace}
