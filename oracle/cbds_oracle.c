/*
 * cbds_oracle.c - CPU oracle of CBDS-P (Section 3.2, Algorithm 2 of De Zoysa
 * et al., "Parallel Algorithms for Densest Subgraph Discovery Using Shared
 * Memory Model"): the densest k-core, extended by "legitimate" outside
 * vertices.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and
 * bench.py's cpu_baseline leg may use this file.  It shares no code with the
 * GPU library.
 *
 * What is computed, in the paper's two phases, with exact integers (every
 * density comparison is a cross-multiplication of int64 counts, done here in
 * 128 bits):
 *
 *  Phase 1 (Algorithm 2, first part).  The core number of every vertex: the
 *  largest k such that the vertex lies in the k-core, the largest subgraph in
 *  which every vertex has degree >= k (Section 2).  The paper reaches it with
 *  the level-synchronous PKC peel; the result is unique, so this oracle uses
 *  the textbook sequential bucket algorithm of Batagelj and Zaversnik, which
 *  removes a vertex of least remaining degree at a time.  For every k the
 *  k-core C_k = { v : core(v) >= k } has |C_k| vertices and |E(C_k)| =
 *  #{edges whose two ends both have core number >= k}.  The densest core is
 *  the non-empty C_K of greatest density; among equal densities the smallest
 *  K wins (the paper scans k upward and updates on a strictly greater
 *  density).  C_0 = G is a candidate.
 *
 *  Phase 2 (Algorithm 2, second part).  rho = |E(C_K)| / |C_K|.  An outside
 *  vertex v (core(v) < K) is eligible when core(v) > rho.  Its count legits(v)
 *  is the number of its neighbours inside C_K; it is legitimate when
 *  legits(v) > rho.  All legitimate vertices L join at once: the result is
 *  S = C_K u L with |E(S)| = |E(C_K)| + sum legits + |E(L)| edges.
 *
 * Readings taken where the printed algorithm is ambiguous (listed in the
 * design notes): the recorded "max_density_core" is the order K of the
 * densest core itself (the printed update records the level k just peeled,
 * whose remaining graph is C_{k+1}); self-edges are outside the input domain.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

enum { CB_OK = 0, CB_EINVAL = -1, CB_ENOMEM = -3 };

/* Core numbers (Batagelj-Zaversnik): vertices in a bucket array ordered by
 * current degree; take a vertex of least degree d, its core number is d; each
 * neighbour of larger current degree loses one and moves one bucket down. */
static int core_numbers(const int32_t* rp, const int32_t* ci, int64_t n, int32_t* core,
                        int32_t* kmax_out) {
    int32_t md = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int32_t d = rp[v + 1] - rp[v];
        core[v] = d;
        if (d > md) md = d;
    }
    int64_t* bin = (int64_t*)calloc((size_t)md + 2, sizeof(int64_t));
    int64_t* pos = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* vert = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!bin || !pos || !vert) {
        free(bin);
        free(pos);
        free(vert);
        return CB_ENOMEM;
    }
    for (int64_t v = 0; v < n; ++v) bin[core[v]]++;
    int64_t start = 0;
    for (int32_t d = 0; d <= md; ++d) {
        const int64_t c = bin[d];
        bin[d] = start;
        start += c;
    }
    for (int64_t v = 0; v < n; ++v) {
        pos[v] = bin[core[v]];
        vert[pos[v]] = v;
        bin[core[v]]++;
    }
    for (int32_t d = md; d >= 1; --d) bin[d] = bin[d - 1];
    bin[0] = 0;
    int32_t kmax = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t v = vert[i];
        if (core[v] > kmax) kmax = core[v];
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int64_t u = ci[e];
            if (core[u] > core[v]) {
                /* swap u with the first vertex of its bucket, shrink the bucket */
                const int32_t du = core[u];
                const int64_t pu = pos[u];
                const int64_t pw = bin[du];
                const int64_t w = vert[pw];
                if (u != w) {
                    pos[u] = pw;
                    vert[pu] = w;
                    pos[w] = pu;
                    vert[pw] = u;
                }
                bin[du]++;
                core[u] = du - 1;
            }
        }
    }
    free(bin);
    free(pos);
    free(vert);
    *kmax_out = kmax;
    return CB_OK;
}

/*
 * out[0..9]: dens_num, dens_den      |E(S)|, |S| of the result S = C_K u L
 *            core_num, core_den      |E(C_K)|, |C_K|
 *            K                       order of the densest core
 *            n_legit                 |L|
 *            kmax                    largest core number
 *            best_size               ids written to best_ids (= |S|)
 *            n_eligible              outside vertices with core(v) > rho
 *            legit_edges             sum of legits over L plus |E(L)|
 * core (n entries) receives the core numbers; best_ids (n entries) S in
 * ascending order.  Returns 0, or a negative code.
 */
int32_t dsg_oracle_cbds(const int32_t* row_ptr, const int32_t* col_idx, int64_t n,
                        int32_t* core, int32_t* best_ids, int64_t* out) {
    if (n < 0 || !out || (n > 0 && (!row_ptr || !core || !best_ids))) return CB_EINVAL;
    memset(out, 0, 10 * sizeof(int64_t));
    if (n == 0) return CB_OK;
    int32_t kmax = 0;
    int rc = core_numbers(row_ptr, col_idx, n, core, &kmax);
    if (rc) return rc;

    /* |C_k| and |E(C_k)| for every k, from histograms of core numbers and of
     * the smaller core number of each edge's two ends */
    int64_t* vcnt = (int64_t*)calloc((size_t)kmax + 2, sizeof(int64_t));
    int64_t* ecnt = (int64_t*)calloc((size_t)kmax + 2, sizeof(int64_t));
    if (!vcnt || !ecnt) {
        free(vcnt);
        free(ecnt);
        return CB_ENOMEM;
    }
    for (int64_t v = 0; v < n; ++v) {
        vcnt[core[v]]++;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int64_t u = col_idx[e];
            if (u > v) ecnt[core[u] < core[v] ? core[u] : core[v]]++;
        }
    }
    for (int32_t k = kmax - 1; k >= 0; --k) {
        vcnt[k] += vcnt[k + 1];
        ecnt[k] += ecnt[k + 1];
    }
    /* densest core: k upward, strict improvement */
    int32_t K = 0;
    int64_t me = ecnt[0], mv = vcnt[0];
    for (int32_t k = 1; k <= kmax; ++k) {
        if (vcnt[k] == 0) break;
        if ((i128)ecnt[k] * mv > (i128)me * vcnt[k]) {
            K = k;
            me = ecnt[k];
            mv = vcnt[k];
        }
    }
    free(vcnt);
    free(ecnt);

    /* phase 2: eligible (K > core(v) > rho) and legitimate (legits > rho) */
    uint8_t* legit = (uint8_t*)calloc((size_t)n, 1);
    if (!legit) return CB_ENOMEM;
    int64_t n_elig = 0, n_legit = 0, sum_legits = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (core[v] >= K || !((i128)core[v] * mv > (i128)me)) continue;
        ++n_elig;
        int64_t legits = 0;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (core[col_idx[e]] >= K) ++legits;
        if ((i128)legits * mv > (i128)me) {
            legit[v] = 1;
            ++n_legit;
            sum_legits += legits;
        }
    }
    int64_t e_l = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (!legit[v]) continue;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int64_t u = col_idx[e];
            if (u > v && legit[u]) ++e_l;
        }
    }
    int64_t cnt = 0;
    for (int64_t v = 0; v < n; ++v)
        if (core[v] >= K || legit[v]) best_ids[cnt++] = (int32_t)v;
    free(legit);
    out[0] = me + sum_legits + e_l;
    out[1] = mv + n_legit;
    out[2] = me;
    out[3] = mv;
    out[4] = K;
    out[5] = n_legit;
    out[6] = kmax;
    out[7] = cnt;
    out[8] = n_elig;
    out[9] = sum_legits + e_l;
    return CB_OK;
}
