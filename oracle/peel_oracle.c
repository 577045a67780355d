/*
 * peel_oracle.c - CPU oracle for Bahmani's (2+2eps)-approximate densest
 * subgraph peeling, in the bulk-synchronous form of P-Bahmani (Algorithm 1,
 * Section 3.1 "Parallelization of Bahmani's Algorithm").
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header or
 * constant with the GPU library; it is plain sequential C written to be
 * checked by eye against the paper.
 *
 * Definitions used (Section 1.2): the edge density of a vertex set S is
 * rho(S) = |E(S)| / |S| with E(S) the edges induced by S (Definition 1); an
 * alpha-approximation returns S~ with rho(S~) >= rho*(G) / alpha
 * (Definition 3); here alpha = 2 + 2 eps.
 *
 * One pass of Algorithm 1, in the paper's order:
 *   part 1   every active vertex whose degree inside the current graph is
 *            at most 2(1+eps) rho fails and leaves the active set;
 *   barrier  (all tests of a pass see the degrees from the pass start);
 *   part 2   for every failed vertex and every neighbour, the neighbour's
 *            degree drops by one and the edge leaves the graph;
 *   reduce   |V| and |E| of the current graph are updated;
 *   keep     if the new density beats the best one seen, the current graph
 *            becomes the answer G~.
 * The loop runs while the current graph has vertices.
 *
 * Readings taken where the paper is silent or inconsistent:
 *   - the test is "<=" and is evaluated exactly, as
 *       deg * |V| * den <= 2 (num + den) * |E|      with eps = num / den,
 *     in 128-bit integers (never in floating point);
 *   - rho is recomputed from |E| and |V| at the start of every pass;
 *   - an edge is removed once: an edge between two vertices that fail in
 *     the same pass is counted twice by the neighbour walk ("intra") and
 *     removed once, so |E| drops by cross + intra / 2 (Definition 1);
 *   - only neighbours still in the graph lose degree;
 *   - the whole graph (pass 0) is a candidate, the empty graph never is, and
 *     the best set is replaced only on a strictly larger density, so the
 *     earliest (largest) set wins a tie;
 *   - "passes" counts every pass including the one that empties the graph.
 *
 * Input: n vertices 0..n-1, symmetric CSR (row_ptr[n+1], col_idx[2m]), no
 * self loops or repeated edges.  dsg_oracle_check_csr() verifies this.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)
#define ORACLE_EINTERNAL (-3)

#define NEVER INT32_MAX /* removal pass of a vertex still in the graph */

typedef struct {
    int64_t dens_num;  /* |E(S~)| */
    int64_t dens_den;  /* |S~|    */
    int32_t passes;    /* passes until the graph is empty */
    int32_t best_pass; /* pass after which S~ was the current graph (0 = G) */
    int64_t best_size; /* |S~| */
} dsg_oracle_result;

typedef struct {
    int64_t s_in;    /* |V| at the start of the pass */
    int64_t e_in;    /* |E| at the start of the pass */
    int64_t thresh;  /* floor(2(num+den)|E| / (|V| den)), reported only */
    int64_t removed; /* failed vertices */
    int64_t cross;   /* walked edges into vertices that stay */
    int64_t intra;   /* walked edges into vertices failing in this pass */
    int64_t scanned; /* adjacency entries walked */
    int64_t s_out;   /* |V| after the pass */
    int64_t e_out;   /* |E| after the pass */
} dsg_oracle_pass;

/* 0 if the CSR is a simple symmetric graph with sorted rows, else < 0. */
int32_t dsg_oracle_check_csr(const int32_t* row_ptr, const int32_t* col_idx, int64_t n) {
    if (n < 0) return ORACLE_EINVAL;
    if (n == 0) return 0;
    if (!row_ptr) return ORACLE_EINVAL;
    if (row_ptr[0] != 0) return -10;
    for (int64_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return -11;
    const int64_t nnz = row_ptr[n];
    if (nnz % 2) return -12;
    if (nnz > 0 && !col_idx) return ORACLE_EINVAL;
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t u = col_idx[e];
            if (u < 0 || u >= n) return -13;
            if (u == v) return -14;
            if (e > row_ptr[v] && col_idx[e - 1] >= u) return -15;
            /* reverse edge present: binary search in row u */
            int64_t lo = row_ptr[u], hi = row_ptr[u + 1];
            int found = 0;
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (col_idx[mid] == v) { found = 1; break; }
                if (col_idx[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (!found) return -16;
        }
    }
    return 0;
}

/*
 * Peel.  removed_at (n entries) receives, for every vertex, the pass in
 * which it failed; best_ids receives S~ in ascending order (room for n);
 * trace receives up to trace_cap pass records.  All three may be NULL.
 */
int32_t dsg_oracle_peel(const int32_t* row_ptr, const int32_t* col_idx, int64_t n,
                        int64_t eps_num, int64_t eps_den, int32_t* removed_at,
                        int32_t* best_ids, dsg_oracle_pass* trace, int64_t trace_cap,
                        dsg_oracle_result* out) {
    if (!out || n < 0 || eps_num < 0 || eps_den < 1) return ORACLE_EINVAL;
    memset(out, 0, sizeof(*out));
    if (n == 0) return ORACLE_OK;
    if (!row_ptr) return ORACLE_EINVAL;

    int32_t* deg = (int32_t*)malloc((size_t)n * sizeof(int32_t));     /* nu.deg */
    int32_t* gone = (int32_t*)malloc((size_t)n * sizeof(int32_t));    /* pass of failure */
    int32_t* failed = (int32_t*)malloc((size_t)n * sizeof(int32_t));  /* failed set */
    if (!deg || !gone || !failed) {
        free(deg); free(gone); free(failed);
        return ORACLE_ENOMEM;
    }

    /* G~ <- G;  |V|, |E| of the current graph */
    int64_t V = n;
    int64_t E = (int64_t)row_ptr[n] / 2;
    for (int64_t v = 0; v < n; ++v) {
        deg[v] = row_ptr[v + 1] - row_ptr[v];
        gone[v] = NEVER;
    }
    int64_t best_E = E, best_V = V;
    int32_t best_pass = 0;
    const __int128 two_one_plus_eps = (__int128)2 * ((__int128)eps_num + eps_den); /* 2(1+eps)*den */

    int32_t pass = 0;
    while (V > 0) {
        ++pass;
        if ((int64_t)pass > n) { /* every valid pass removes a vertex */
            free(deg); free(gone); free(failed);
            return ORACLE_EINTERNAL;
        }
        const int64_t V_in = V, E_in = E;

        /* part 1: active vertices with deg <= 2(1+eps) rho fail */
        int64_t n_failed = 0;
        for (int64_t v = 0; v < n; ++v) {
            if (gone[v] != NEVER) continue; /* not active */
            const __int128 lhs = (__int128)deg[v] * V_in * eps_den;
            const __int128 rhs = two_one_plus_eps * E_in;
            if (lhs <= rhs) {
                failed[n_failed++] = (int32_t)v;
                gone[v] = pass;
            }
        }
        /* barrier: every failure of this pass is known before part 2 */

        /* part 2: walk the neighbours of every failed vertex */
        int64_t cross = 0, intra = 0, scanned = 0;
        for (int64_t i = 0; i < n_failed; ++i) {
            const int32_t v = failed[i];
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                const int32_t u = col_idx[e];
                ++scanned;
                if (gone[u] == NEVER) {
                    deg[u] -= 1; /* atomicSub(u.deg, 1) */
                    ++cross;
                } else if (gone[u] == pass) {
                    ++intra; /* both ends fail now: seen from each end */
                }
            }
        }
        if (n_failed == 0 || (intra & 1)) {
            free(deg); free(gone); free(failed);
            return ORACLE_EINTERNAL;
        }

        /* reduce */
        V -= n_failed;
        E -= cross + intra / 2;
        if (E < 0 || (V == 0 && E != 0)) {
            free(deg); free(gone); free(failed);
            return ORACLE_EINTERNAL;
        }

        if (trace && (int64_t)(pass - 1) < trace_cap) {
            dsg_oracle_pass* t = &trace[pass - 1];
            t->s_in = V_in;
            t->e_in = E_in;
            t->thresh = (int64_t)((two_one_plus_eps * E_in) / ((__int128)V_in * eps_den));
            t->removed = n_failed;
            t->cross = cross;
            t->intra = intra;
            t->scanned = scanned;
            t->s_out = V;
            t->e_out = E;
        }

        /* keep the denser graph: E / V > best_E / best_V */
        if (V > 0 && (__int128)E * best_V > (__int128)best_E * V) {
            best_E = E;
            best_V = V;
            best_pass = pass;
        }
    }

    /* G~ is the graph left after pass best_pass */
    int64_t k = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (gone[v] > best_pass) {
            if (best_ids) best_ids[k] = (int32_t)v;
            ++k;
        }
        if (removed_at) removed_at[v] = gone[v];
    }
    free(deg); free(gone); free(failed);
    if (k != best_V) return ORACLE_EINTERNAL;

    out->dens_num = best_E;
    out->dens_den = best_V;
    out->passes = pass;
    out->best_pass = best_pass;
    out->best_size = best_V;
    return ORACLE_OK;
}
