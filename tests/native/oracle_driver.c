/*
 * oracle_driver.c - runs the C oracles (oracle/peel_oracle.c and
 * oracle/cbds_oracle.c) over generated graphs and over inputs that break
 * the CSR contract, for a build with the address and undefined-behaviour
 * sanitizers.  Test infrastructure only: a memory or arithmetic error aborts
 * the run; otherwise it checks a few identities of Algorithm 1 (Section 3.1)
 * and prints "ok".
 *
 * Exit status: 0 when every check held, 1 otherwise.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t dens_num, dens_den;
    int32_t passes, best_pass;
    int64_t best_size;
} res_t;

typedef struct {
    int64_t s_in, e_in, thresh, removed, cross, intra, scanned, s_out, e_out;
} pass_t;

int32_t dsg_oracle_check_csr(const int32_t* row_ptr, const int32_t* col_idx, int64_t n);
int32_t dsg_oracle_peel(const int32_t* row_ptr, const int32_t* col_idx, int64_t n,
                        int64_t eps_num, int64_t eps_den, int32_t* removed_at, int32_t* best_ids,
                        pass_t* trace, int64_t trace_cap, res_t* out);
int32_t dsg_oracle_cbds(const int32_t* row_ptr, const int32_t* col_idx, int64_t n, int32_t* core,
                        int32_t* best_ids, int64_t* out);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void) { /* xorshift64* */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 2685821657736338717ull;
}

static int failures = 0;
#define CHECK(c, ...)                                   \
    do {                                                \
        if (!(c)) {                                     \
            fprintf(stderr, "check failed: " __VA_ARGS__); \
            fputc('\n', stderr);                        \
            ++failures;                                 \
        }                                               \
    } while (0)

/* symmetric CSR of an n-vertex graph whose upper-triangle adjacency is
 * adj[u * n + v] (u < v); rows ascending */
static void build_csr(int n, const uint8_t* adj, int32_t** rp, int32_t** ci) {
    int32_t* r = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
    int64_t nnz = 0;
    for (int u = 0; u < n; ++u)
        for (int v = 0; v < n; ++v)
            if (u != v && adj[u < v ? u * n + v : v * n + u]) ++nnz;
    int32_t* c = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    int64_t k = 0;
    for (int u = 0; u < n; ++u) {
        r[u] = (int32_t)k;
        for (int v = 0; v < n; ++v)
            if (u != v && adj[u < v ? u * n + v : v * n + u]) c[k++] = v;
    }
    r[n] = (int32_t)k;
    *rp = r;
    *ci = c;
}

static void run_valid(int n, const int32_t* rp, const int32_t* ci) {
    static const int64_t eps[][2] = {{0, 1}, {1, 100}, {1, 10}, {1, 2}, {1, 1}, {3, 1}};
    CHECK(dsg_oracle_check_csr(rp, ci, n) == 0, "valid csr rejected (n=%d)", n);
    int32_t* rem = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t* best = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    pass_t* tr = (pass_t*)malloc(((size_t)n + 1) * sizeof(pass_t));
    for (int e = 0; e < 6; ++e) {
        res_t r;
        const int32_t rc = dsg_oracle_peel(rp, ci, n, eps[e][0], eps[e][1], rem, best, tr, n + 1, &r);
        CHECK(rc == 0, "peel failed (n=%d rc=%d)", n, rc);
        if (rc) continue;
        int64_t removed = 0, scanned = 0, edges = 0;
        for (int32_t k = 0; k < r.passes; ++k) {
            removed += tr[k].removed;
            scanned += tr[k].scanned;
            edges += tr[k].cross + tr[k].intra / 2;
            CHECK(tr[k].intra % 2 == 0, "odd intra");
        }
        CHECK(removed == n && r.passes <= n, "removal count (n=%d)", n);
        CHECK(scanned == rp[n] && 2 * edges == rp[n], "edge accounting (n=%d)", n);
        CHECK(r.best_size == r.dens_den, "best size");
        int64_t kept = 0;
        for (int v = 0; v < n; ++v) kept += rem[v] > r.best_pass;
        CHECK(kept == r.dens_den, "best set");
    }
    int64_t out[10];
    const int32_t rc = dsg_oracle_cbds(rp, ci, n, rem, best, out);
    CHECK(rc == 0, "cbds failed (n=%d rc=%d)", n, rc);
    if (rc == 0) {
        CHECK(out[7] == out[1], "cbds result size");
        CHECK(out[2] * 1 <= out[0] && out[3] <= out[1], "cbds extension only adds");
    }
    free(rem);
    free(best);
    free(tr);
}

/* a CSR whose vertices 1..10 list vertex 0 while 0 lists only 1 and 2:
 * pass 1 removes 1..10 and takes ten decrements off a degree of 2, so the
 * edge count goes negative and the oracle stops with its internal error */
static void run_one_sided(void) {
    const int32_t rp[12] = {0, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12};
    const int32_t ci[12] = {1, 2, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    int32_t rem[11], best[11];
    pass_t tr[12];
    res_t r;
    CHECK(dsg_oracle_check_csr(rp, ci, 11) == -16, "one-sided rows not rejected");
    CHECK(dsg_oracle_peel(rp, ci, 11, 1, 10, rem, best, tr, 12, &r) == -3,
          "one-sided rows not an internal error");
}

int main(int argc, char** argv) {
    const int graphs = argc > 1 ? atoi(argv[1]) : 300;
    int64_t runs = 0, broken_ok = 0;
    for (int gi = 0; gi < graphs; ++gi) {
        const int n = (int)(rnd() % 120);
        const uint64_t p = rnd() % 1000; /* edge probability in 1/1000 */
        uint8_t* adj = (uint8_t*)calloc((size_t)n * n + 1, 1);
        for (int u = 0; u < n; ++u)
            for (int v = u + 1; v < n; ++v) adj[u * n + v] = (uint8_t)(rnd() % 1000 < p);
        int32_t *rp, *ci;
        build_csr(n, adj, &rp, &ci);
        run_valid(n, rp, ci);
        ++runs;
        /* the same rows with some entries overwritten by another in-range
         * id: duplicates, self loops or one-sided edges, whatever comes out.
         * The checker rejects it; the peel must end (any status) without a
         * memory or arithmetic error */
        if (rp[n] > 0) {
            const int hits = 1 + (int)(rnd() % 4);
            for (int h = 0; h < hits; ++h) ci[rnd() % (uint64_t)rp[n]] = (int32_t)(rnd() % (uint64_t)n);
            int32_t* rem = (int32_t*)malloc((size_t)n * sizeof(int32_t));
            int32_t* best = (int32_t*)malloc((size_t)n * sizeof(int32_t));
            pass_t* tr = (pass_t*)malloc(((size_t)n + 1) * sizeof(pass_t));
            res_t r;
            const int32_t rc = dsg_oracle_peel(rp, ci, n, 1, 10, rem, best, tr, n + 1, &r);
            broken_ok += rc == 0 || rc == -3;
            CHECK(rc == 0 || rc == -3, "broken csr: unexpected status %d", rc);
            free(rem);
            free(best);
            free(tr);
        }
        free(adj);
        free(rp);
        free(ci);
    }
    run_one_sided();
    /* the empty graph and a null graph */
    {
        const int32_t rp0[1] = {0};
        res_t r;
        CHECK(dsg_oracle_peel(rp0, NULL, 0, 1, 10, NULL, NULL, NULL, 0, &r) == 0 && r.passes == 0,
              "n = 0");
        CHECK(dsg_oracle_peel(NULL, NULL, 3, 1, 10, NULL, NULL, NULL, 0, &r) == -1, "null rows");
        CHECK(dsg_oracle_peel(rp0, NULL, 0, 1, 0, NULL, NULL, NULL, 0, &r) == -1, "den 0");
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok %lld graphs, %lld broken inputs ended cleanly\n", (long long)runs,
           (long long)broken_ok);
    return 0;
}
