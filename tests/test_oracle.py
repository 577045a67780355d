"""Pins for the CPU oracle (no GPU).

The oracle is checked against things it does not compute itself:
hand-derived worked examples (tests/golden), a literal re-statement that
recomputes every degree and edge count from Definition 1 in each pass, exact
densest-subgraph densities (brute force and Goldberg max-flow) for the
(2+2eps) guarantee of Section 3.1, the O(log_{1+eps} n) pass bound, edge
accounting identities, closed forms and relabelling invariance.  The last
block plants plausible mistakes in a copy of the literal oracle and checks
that these pins reject each of them.
"""
from __future__ import annotations

import itertools
import random

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import exact, literal
from paper_2103_00154_amd import inputs

EPS = [(0, 1), (1, 100), (1, 10), (1, 2), (1, 1), (3, 1)]


def _c(g, e):
    return oracle.peel_graph(g, *e)


def _edges(g):
    return [tuple(map(int, x)) for x in g.edges()]


# ---------------------------------------------------------------- golden

def test_golden_c_oracle(golden):
    for case in golden:
        g = inputs.from_edges(case["n"], case["edges"])
        r = oracle.peel_graph(g, *case["eps"])
        x = case["expect"]
        assert (r.passes, r.best_pass, r.num, r.den) == (
            x["passes"], x["best_pass"], x["num"], x["den"]), case["name"]
        assert r.best.tolist() == x["best"], case["name"]
        if "removed_at" in x:
            assert r.removed_at.tolist() == x["removed_at"], case["name"]
        for got, want in zip(r.trace, x.get("trace", [])):
            for k, v in want.items():
                assert got[k] == v, (case["name"], k)


def test_golden_literal(golden):
    for case in golden:
        r = literal.peel_literal(case["n"], case["edges"], *case["eps"])
        x = case["expect"]
        assert (r["passes"], r["best_pass"], r["num"], r["den"]) == (
            x["passes"], x["best_pass"], x["num"], x["den"]), case["name"]
        assert r["best"] == x["best"], case["name"]


# ------------------------------------------------- C oracle == literal oracle

def _same(g, e):
    c = _c(g, e)
    lit = literal.peel_literal(g.n, _edges(g), *e)
    assert c.passes == lit["passes"]
    assert c.best_pass == lit["best_pass"]
    assert (c.num, c.den) == (lit["num"], lit["den"])
    assert c.best.tolist() == lit["best"]
    assert c.removed_at.tolist() == lit["removed_at"]
    assert c.trace == lit["trace"]
    return c


def _all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield inputs.from_edges(n, [p for i, p in enumerate(pairs) if mask >> i & 1])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_tiny_graphs_match_literal(n):
    for g in _all_graphs(n):
        for e in EPS:
            _same(g, e)


def test_sampled_six_and_seven_vertex_graphs_match_literal():
    rnd = random.Random(6)
    for n in (6, 7):
        pairs = list(itertools.combinations(range(n), 2))
        for _ in range(400):
            mask = rnd.getrandbits(len(pairs))
            g = inputs.from_edges(n, [p for i, p in enumerate(pairs) if mask >> i & 1])
            _same(g, rnd.choice(EPS))


def _literal_all(n, eps_num, eps_den):
    """Definition 1 and Algorithm 1 over every labelled graph on n vertices
    at once: graph i has edge j of itertools.combinations(range(n), 2) iff
    bit j of i is set.  Every pass recounts deg_S(v) = |N(v) & S| and |E(S)|
    from the edge bits (no running counts).  Returns per-graph arrays."""
    pairs = list(itertools.combinations(range(n), 2))
    G = 1 << len(pairs)
    gid = np.arange(G, dtype=np.int64)
    has = np.stack([(gid >> j) & 1 for j in range(len(pairs))]).astype(bool)  # [pair, graph]
    inS = np.ones((n, G), dtype=bool)

    def deg_in(members):  # |N(v) & members| for every v, every graph
        d = np.zeros((n, G), dtype=np.int64)
        for j, (u, v) in enumerate(pairs):
            d[u] += has[j] & members[v]
            d[v] += has[j] & members[u]
        return d

    def edges_in(members):
        e = np.zeros(G, dtype=np.int64)
        for j, (u, v) in enumerate(pairs):
            e += has[j] & members[u] & members[v]
        return e

    removed_at = np.full((n, G), oracle.NEVER, dtype=np.int64)
    best_e, best_v = edges_in(inS), np.full(G, n, dtype=np.int64)
    best_pass = np.zeros(G, dtype=np.int64)
    passes = np.zeros(G, dtype=np.int64)
    trace = []  # per pass: dict of [graph] arrays (entries of finished graphs unused)
    for k in range(1, n + 1):
        live = inS.any(axis=0)
        if not live.any():
            break
        V = inS.sum(axis=0)
        E = edges_in(inS)
        d = deg_in(inS)
        failed = inS & (d * V * eps_den <= 2 * (eps_num + eps_den) * E)
        nxt = inS & ~failed
        E_next = edges_in(nxt)
        full = deg_in(np.ones((n, G), dtype=bool))
        trace.append({
            "s_in": V, "e_in": E,
            "thresh": np.where(V > 0, (2 * (eps_num + eps_den) * E) // np.maximum(V * eps_den, 1), 0),
            "removed": failed.sum(axis=0),
            "cross": (deg_in(nxt) * failed).sum(axis=0),
            "intra": (deg_in(failed) * failed).sum(axis=0),
            "scanned": (full * failed).sum(axis=0),
            "s_out": nxt.sum(axis=0), "e_out": E_next, "live": live})
        removed_at[failed] = k
        passes[live] = k
        V_next = nxt.sum(axis=0)
        better = live & (V_next > 0) & (E_next * best_v > best_e * V_next)
        best_e = np.where(better, E_next, best_e)
        best_v = np.where(better, V_next, best_v)
        best_pass = np.where(better, k, best_pass)
        inS = nxt
    return {"passes": passes, "best_pass": best_pass, "num": best_e, "den": best_v,
            "removed_at": removed_at, "trace": trace, "pairs": pairs}


def test_vectorised_literal_equals_the_literal_oracle():
    # the all-graphs form of the literal oracle against its plain form
    for n in (3, 4):
        for e in EPS:
            a = _literal_all(n, *e)
            pairs = a["pairs"]
            for i in range(1 << len(pairs)):
                lit = literal.peel_literal(n, [p for j, p in enumerate(pairs) if i >> j & 1], *e)
                assert (lit["passes"], lit["best_pass"], lit["num"], lit["den"]) == (
                    a["passes"][i], a["best_pass"][i], a["num"][i], a["den"][i])
                assert lit["removed_at"] == a["removed_at"][:, i].tolist()
                for k, t in enumerate(lit["trace"]):
                    for f, v in t.items():
                        assert a["trace"][k][f][i] == v, (n, e, i, k, f)


@pytest.mark.parametrize("e", EPS)
def test_exhaustive_six_vertex_graphs_match_literal(e):
    # every labelled graph on six vertices (2^15 of them), C oracle against
    # the literal restatement, every field and every pass
    n = 6
    a = _literal_all(n, *e)
    pairs = a["pairs"]
    rows = [[u for u in range(n) if u != v] for v in range(n)]
    pair_index = {p: j for j, p in enumerate(pairs)}
    for i in range(1 << len(pairs)):
        rp, ci = [0], []
        for v in range(n):
            ci += [u for u in rows[v] if i >> pair_index[(min(u, v), max(u, v))] & 1]
            rp.append(len(ci))
        c = oracle.peel(np.array(rp, np.int32), np.array(ci, np.int32), n, *e)
        assert (c.passes, c.best_pass, c.num, c.den) == (
            a["passes"][i], a["best_pass"][i], a["num"][i], a["den"][i]), (e, i)
        assert c.removed_at.tolist() == a["removed_at"][:, i].tolist(), (e, i)
        assert c.best.tolist() == [v for v in range(n) if a["removed_at"][v, i] > c.best_pass]
        for k, t in enumerate(c.trace):
            for f, v in t.items():
                assert a["trace"][k][f][i] == v, (e, i, k, f)


@st.composite
def _hyp_graphs(draw, max_n=12):
    """A graph on 1..max_n vertices with any edge set (each possible edge
    drawn independently), plus an eps from the tested set."""
    n = draw(st.integers(1, max_n))
    pairs = list(itertools.combinations(range(n), 2))
    keep = draw(st.lists(st.booleans(), min_size=len(pairs), max_size=len(pairs)))
    e = draw(st.sampled_from(EPS))
    return n, [p for p, k in zip(pairs, keep) if k], e


@settings(max_examples=400, deadline=None, derandomize=True)
@given(_hyp_graphs())
def test_hypothesis_graphs_match_literal(case):
    # property-based: hypothesis searches edge sets (and shrinks any failure
    # to a smallest graph); derandomized, so every run checks the same cases
    n, edges, e = case
    _same(inputs.from_edges(n, edges), e)


@pytest.mark.parametrize("seed", range(40))
def test_random_graphs_up_to_40_vertices_match_literal(seed):
    rnd = random.Random(seed)
    n = rnd.randint(5, 40)
    g = inputs.random_small(n, rnd.choice([0.05, 0.15, 0.3, 0.6]), seed)
    _same(g, rnd.choice(EPS))


# ------------------------------------------- approximation guarantee (Def. 3)

def _guarantee(c, e_star, s_star, e):
    num, den = e
    # rho(S~) >= rho* / (2 + 2 eps)  <=>  2 (num+den) E(S~) |S*| >= den E(S*) |S~|
    assert 2 * (num + den) * c.num * s_star >= den * e_star * c.den


@pytest.mark.parametrize("seed", range(60))
def test_guarantee_against_bruteforce(seed):
    rnd = random.Random(1000 + seed)
    n = rnd.randint(2, 12)
    g = inputs.random_small(n, rnd.choice([0.2, 0.35, 0.5, 0.8]), seed)
    e_star, s_star, _ = exact.densest_bruteforce(n, _edges(g))
    for e in EPS:
        _guarantee(_c(g, e), e_star, s_star, e)


@pytest.mark.parametrize("seed", range(25))
def test_goldberg_matches_bruteforce(seed):
    rnd = random.Random(2000 + seed)
    n = rnd.randint(1, 12)
    g = inputs.random_small(n, rnd.choice([0.15, 0.3, 0.5, 0.9]), seed)
    eb, sb, _ = exact.densest_bruteforce(n, _edges(g))
    eg, sg, mask = exact.densest_goldberg(n, _edges(g))
    assert eb * sg == eg * sb
    # the returned set really has that density
    members = set(np.flatnonzero(mask).tolist())
    assert sum(1 for u, v in _edges(g) if u in members and v in members) == eg
    assert len(members) == sg


def _densest_union_bruteforce(n, edges):
    """rho* and the union of every subset of density rho* (brute force)."""
    adj = [0] * n
    for u, v in edges:
        adj[u] |= 1 << v
        adj[v] |= 1 << u
    best, union = (0, 1), 0
    for mask in range(1, 1 << n):
        size = bin(mask).count("1")
        e = sum(bin(adj[v] & mask).count("1") for v in range(n) if mask >> v & 1) // 2
        if e * best[1] > best[0] * size:
            best, union = (e, size), mask
        elif e * best[1] == best[0] * size:
            union |= mask
    return best, [v for v in range(n) if union >> v & 1]


@pytest.mark.parametrize("seed", range(40))
def test_maximal_densest_matches_bruteforce_union(seed):
    rnd = random.Random(3000 + seed)
    n = rnd.randint(1, 11)
    g = inputs.random_small(n, rnd.choice([0.15, 0.3, 0.5, 0.9]), seed)
    (eb, sb), union = _densest_union_bruteforce(n, _edges(g))
    e, s, mask = exact.densest_maximal(n, _edges(g))
    assert e * sb == eb * s
    assert np.flatnonzero(mask).tolist() == union
    assert sum(1 for u, v in _edges(g) if mask[u] and mask[v]) == e and int(mask.sum()) == s


def test_maximal_densest_closed_forms():
    # two equal cliques: both are densest, so is their union
    e, s, mask = exact.densest_maximal(12, _edges(inputs.disjoint_cliques(6, 6)))
    assert (e, s) == (30, 12)
    e, s, mask = exact.densest_maximal(10, _edges(inputs.disjoint_cliques(6, 4)))
    assert (e, s) == (15, 6) and np.flatnonzero(mask).tolist() == list(range(6))
    e, s, mask = exact.densest_maximal(7, [])
    assert (e, s) == (0, 7)
    g = inputs.star(30)  # k leaves: k / (k + 1) beats every proper subset
    assert exact.densest_maximal(g.n, _edges(g))[:2] == (29, 30)


def _medium_graphs():
    yield inputs.erdos_renyi(400, 2000, 0)
    yield inputs.rmat(9, 8, seed=3)
    yield inputs.chung_lu(600, 12, 2.3, 5)
    yield inputs.rmat(10, 4, seed=1, planted=(40, 0.6, 2))
    yield inputs.disjoint_cliques(30, 12)


@pytest.mark.parametrize("gi", range(5))
def test_guarantee_against_goldberg(gi):
    g = list(_medium_graphs())[gi]
    e_star, s_star, _ = exact.densest_goldberg(g.n, _edges(g))
    for e in EPS:
        _guarantee(_c(g, e), e_star, s_star, e)


@pytest.mark.parametrize("gi", range(5))
def test_maximal_densest_density_equals_goldberg(gi):
    g = list(_medium_graphs())[gi]
    e1, s1, _ = exact.densest_goldberg(g.n, _edges(g))
    e2, s2, mask = exact.densest_maximal(g.n, _edges(g))
    assert e1 * s2 == e2 * s1
    assert int(mask.sum()) >= s1  # the largest densest subgraph


def test_planted_block_density_is_reached():
    g = inputs.rmat(11, 4, seed=7, planted=(60, 0.7, 1))
    ids = set(g.meta["planted_ids"].tolist())
    e_p = sum(1 for u, v in _edges(g) if u in ids and v in ids)
    for e in [(1, 10), (1, 1)]:
        c = _c(g, e)
        num, den = e
        assert 2 * (num + den) * c.num * len(ids) >= den * e_p * c.den


# --------------------------------------------------------- pass bound etc.

def _pass_bound(n, num, den):
    """Least K >= 1 with (num+den)^K >= n den^K, or n when eps = 0."""
    if n <= 1:
        return n
    if num == 0:
        return n
    k, a, b = 1, num + den, den
    while a < n * b:
        k += 1
        a *= num + den
        b *= den
    return k


def _graph_zoo():
    yield inputs.erdos_renyi(10000, 50000, 0)
    yield inputs.rmat(12, 16, seed=0)
    yield inputs.chung_lu(3000, 20, 2.1, 1)
    yield inputs.star(500)
    yield inputs.path(300)
    yield inputs.disjoint_cliques(20, 7)
    yield inputs.empty(50)


@pytest.mark.parametrize("e", EPS)
def test_pass_bound_and_shrink_invariant(e):
    num, den = e
    for g in _graph_zoo():
        c = _c(g, e)
        assert c.passes <= _pass_bound(g.n, num, den), g.name
        for t in c.trace:
            # survivors all have degree above the threshold, so
            # |S_k| (num+den) < |S_{k-1}| den unless S_k is empty
            assert t["s_out"] == 0 or t["s_out"] * (num + den) < t["s_in"] * den


@pytest.mark.parametrize("e", EPS)
def test_edge_accounting(e):
    for g in _graph_zoo():
        c = _c(g, e)
        assert sum(t["removed"] for t in c.trace) == g.n
        assert sum(t["scanned"] for t in c.trace) == 2 * g.m
        assert all(t["intra"] % 2 == 0 for t in c.trace)
        assert sum(t["cross"] + t["intra"] // 2 for t in c.trace) == g.m
        for a, b in zip(c.trace, c.trace[1:]):
            assert (b["s_in"], b["e_in"]) == (a["s_out"], a["e_out"])
        # removal passes match the trace and S~ is what survived best_pass
        counts = np.bincount(c.removed_at, minlength=c.passes + 1)[1:]
        assert counts.tolist() == [t["removed"] for t in c.trace]
        assert c.best.tolist() == np.flatnonzero(c.removed_at > c.best_pass).tolist()


def test_edge_count_recomputed_from_survivors():
    g = inputs.rmat(11, 8, seed=2)
    c = _c(g, (1, 10))
    e = g.edges()
    for k, t in enumerate(c.trace, start=1):
        alive = c.removed_at > k
        assert int(np.count_nonzero(alive[e[:, 0]] & alive[e[:, 1]])) == t["e_out"]
        assert int(alive.sum()) == t["s_out"]


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("g", [inputs.clique(7), inputs.cycle(11), inputs.empty(4),
                               inputs.from_edges(8, [(i, (i + 1) % 8) for i in range(8)]
                                                 + [(i, (i + 4) % 8) for i in range(4)])])
def test_regular_graphs_one_pass(g):
    for e in EPS:
        c = _c(g, e)
        assert (c.passes, c.best_pass, c.num, c.den) == (1, 0, g.m, g.n)


def test_large_eps_single_pass():
    g = inputs.chung_lu(2000, 16, 2.2, 3)
    maxdeg = int(g.degrees().max())
    den = 7
    num = -(-maxdeg * g.n * den // (2 * g.m)) - den  # smallest with 2(num+den)m >= maxdeg n den
    assert 2 * (num + den) * g.m >= maxdeg * g.n * den
    c = _c(g, (num, den))
    assert (c.passes, c.best_pass, c.num, c.den) == (1, 0, g.m, g.n)


@pytest.mark.parametrize("a,b", [(6, 3), (9, 4), (12, 8)])
def test_disjoint_cliques_recover_larger(a, b):
    g = inputs.disjoint_cliques(a, b)
    num, den = 1, 10
    t1 = 2 * (num + den) * g.m // (g.n * den)
    assert b - 1 <= t1 < a - 1
    c = _c(g, (num, den))
    assert c.best.tolist() == list(range(a))
    assert (c.num, c.den) == (a * (a - 1) // 2, a)


def test_relabel_permutes_result():
    g = inputs.chung_lu(1500, 10, 2.4, 9)
    perm = np.random.default_rng(4).permutation(g.n)
    h = inputs.relabel(g, perm)
    for e in [(1, 10), (0, 1)]:
        a, b = _c(g, e), _c(h, e)
        assert (a.passes, a.best_pass, a.num, a.den) == (b.passes, b.best_pass, b.num, b.den)
        assert sorted(perm[a.best].tolist()) == b.best.tolist()
        assert np.array_equal(b.removed_at[perm], a.removed_at)
        assert a.trace == b.trace


# ------------------------------------------------------------ input checks

def test_argument_errors():
    g = inputs.path(3)
    for bad in [(0, 0), (-1, 1), (1, -5)]:
        with pytest.raises(oracle.OracleError):
            oracle.peel_graph(g, *bad)


def test_check_csr():
    g = inputs.rmat(8, 4, seed=1)
    assert oracle.check_csr(g.row_ptr, g.col_idx, g.n) == 0
    ci = g.col_idx.copy()
    ci[0], ci[1] = ci[1], ci[0]  # unsorted row
    assert oracle.check_csr(g.row_ptr, ci, g.n) != 0
    one_way = inputs.Graph(n=3, m=1, row_ptr=np.array([0, 1, 1, 2], np.int32),
                           col_idx=np.array([1, 1], np.int32))
    assert oracle.check_csr(one_way.row_ptr, one_way.col_idx, 3) != 0


# ------------------------------------------------- pins reject planted bugs

def _mutant(n, edges, num, den, bug, cap=200):
    """Copy of the literal oracle with one planted mistake."""
    edges = [(min(u, v), max(u, v)) for u, v in edges]
    adj = {v: set() for v in range(n)}
    for u, v in edges:
        adj[u].add(v)
        adj[v].add(u)
    S = set(range(n))
    removed = [None] * n
    E = len(edges)
    best = (E, n, 0)
    k = 0
    while S and k < cap:
        k += 1
        V = len(S)
        if bug == "strict":
            fail = {v for v in S if len(adj[v] & S) * V * den < 2 * (num + den) * E}
        elif bug == "no_factor_two":
            fail = {v for v in S if len(adj[v] & S) * V * den <= (num + den) * E}
        else:
            fail = {v for v in S if len(adj[v] & S) * V * den <= 2 * (num + den) * E}
        for v in fail:
            removed[v] = k
        nxt = S - fail
        if bug == "charge_every_entry":
            E -= sum(len(adj[v] & S) for v in fail)
        else:
            E = sum(1 for u, v in edges if u in nxt and v in nxt)
        if nxt and (E * best[1] >= best[0] * len(nxt) if bug == "ties_later"
                    else E * best[1] > best[0] * len(nxt)):
            best = (E, len(nxt), k)
        S = nxt
    return {"passes": k, "best_pass": best[2], "num": best[0], "den": best[1]}


@pytest.mark.parametrize("bug", ["strict", "no_factor_two", "charge_every_entry", "ties_later"])
def test_golden_rejects_planted_mistakes(golden, bug):
    caught = False
    for case in golden:
        r = _mutant(case["n"], case["edges"], *case["eps"], bug=bug)
        x = case["expect"]
        if (r["passes"], r["best_pass"], r["num"], r["den"]) != (
                x["passes"], x["best_pass"], x["num"], x["den"]):
            caught = True
    assert caught, f"worked examples do not detect the '{bug}' mistake"
