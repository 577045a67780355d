/*
 * graphgen.c - seeded synthetic undirected graphs in CSR form.
 *
 * This file produces INPUTS only.  It holds none of the peeling arithmetic:
 * both the CPU oracle and the GPU library are fed from what it builds, so it
 * must not know anything about densities, thresholds or passes.
 *
 * Randomness is counter based: draw(base, i) is a pure function of a stream
 * base and a counter, so every generator is deterministic and independent of
 * the number of OpenMP threads.  The mixing function is the SplitMix64
 * finaliser (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014), used as a counter-mode hash.
 *
 * Edges are exchanged as 64-bit directed keys (row << 32 | col).  Every
 * generator emits both directions of each undirected edge; self loops are
 * written as GG_NONE and are removed together with duplicates by
 * gg_sort_unique().  gg_keys_to_csr() then turns the sorted unique keys into
 * int32 row_ptr / col_idx with ascending neighbours in every row.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define GG_NONE UINT64_MAX

static inline uint64_t gg_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Base of stream `stream` under `seed`. */
static inline uint64_t gg_base(uint64_t seed, uint64_t stream) {
    return gg_mix(gg_mix(seed + 0x9E3779B97F4A7C15ULL) ^ (stream * 0xD1B54A32D192ED03ULL));
}

/* The i-th 64-bit draw of a stream. */
static inline uint64_t gg_draw(uint64_t base, uint64_t i) {
    return gg_mix(base + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

/* Uniform integer in [0, n) from a 64-bit draw (multiply-shift). */
static inline uint64_t gg_below(uint64_t r, uint64_t n) {
    return (uint64_t)(((unsigned __int128)r * n) >> 64);
}

static inline uint64_t gg_key(uint64_t r, uint64_t c) { return (r << 32) | c; }

uint64_t gg_draw_for_test(uint64_t seed, uint64_t stream, uint64_t i) {
    return gg_draw(gg_base(seed, stream), i);
}

/* ------------------------------------------------------------------ */
/* R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004).                      */
/* Sample i picks one quadrant per level, most significant bit first,   */
/* from a 32-bit uniform u: u < ta -> (0,0), u < tab -> (0,1),          */
/* u < tabc -> (1,0), else (1,1).  Two levels per 64-bit draw.          */
/* Writes keys[2i], keys[2i+1]; returns nsamples*2.                     */
/* ------------------------------------------------------------------ */
int64_t gg_rmat_keys(int32_t scale, int64_t nsamples, uint64_t ta, uint64_t tab,
                     uint64_t tabc, uint64_t seed, uint64_t stream, uint64_t* keys) {
    if (scale < 1 || scale > 30 || nsamples < 0) return -1;
    const uint64_t base = gg_base(seed, stream);
    const int32_t draws = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nsamples; ++i) {
        uint64_t r = 0, c = 0;
        uint64_t word = 0;
        for (int32_t lvl = 0; lvl < scale; ++lvl) {
            if ((lvl & 1) == 0) word = gg_draw(base, (uint64_t)i * (uint64_t)draws + (uint64_t)(lvl >> 1));
            const uint64_t u = (lvl & 1) ? (word >> 32) : (word & 0xFFFFFFFFULL);
            const uint64_t bit = 1ULL << (scale - 1 - lvl);
            if (u < ta) {
            } else if (u < tab) {
                c |= bit;
            } else if (u < tabc) {
                r |= bit;
            } else {
                r |= bit;
                c |= bit;
            }
        }
        if (r == c) {
            keys[2 * i] = GG_NONE;
            keys[2 * i + 1] = GG_NONE;
        } else {
            keys[2 * i] = gg_key(r, c);
            keys[2 * i + 1] = gg_key(c, r);
        }
    }
    return 2 * nsamples;
}

/* ------------------------------------------------------------------ */
/* Small open-addressing set of uint64 keys (never holds GG_NONE).      */
/* ------------------------------------------------------------------ */
typedef struct { uint64_t* slot; uint64_t mask; } gg_set;

static int gg_set_init(gg_set* s, uint64_t expect) {
    uint64_t cap = 16;
    while (cap < 2 * expect + 16) cap <<= 1;
    s->slot = (uint64_t*)malloc(cap * sizeof(uint64_t));
    if (!s->slot) return -1;
    memset(s->slot, 0xFF, cap * sizeof(uint64_t));
    s->mask = cap - 1;
    return 0;
}

/* returns 1 if inserted, 0 if present */
static int gg_set_insert(gg_set* s, uint64_t k) {
    uint64_t h = gg_mix(k) & s->mask;
    for (;;) {
        if (s->slot[h] == GG_NONE) { s->slot[h] = k; return 1; }
        if (s->slot[h] == k) return 0;
        h = (h + 1) & s->mask;
    }
}

/* ------------------------------------------------------------------ */
/* Erdos-Renyi G(n, m): uniform ordered pairs drawn in counter order;   */
/* loops and repeats of an already drawn edge are rejected until m      */
/* distinct edges exist.  Writes 2m keys; returns 2m, or -1 on bad args.*/
/* ------------------------------------------------------------------ */
int64_t gg_er_keys(int64_t n, int64_t m, uint64_t seed, uint64_t stream, uint64_t* keys) {
    if (n < 0 || m < 0) return -1;
    if (n < 2) return m == 0 ? 0 : -1;
    if ((unsigned __int128)m * 2 > (unsigned __int128)n * (uint64_t)(n - 1)) return -1;
    gg_set set;
    if (gg_set_init(&set, (uint64_t)m)) return -1;
    const uint64_t base = gg_base(seed, stream);
    int64_t have = 0;
    uint64_t ctr = 0;
    while (have < m) {
        const uint64_t u = gg_below(gg_draw(base, ctr++), (uint64_t)n);
        const uint64_t v = gg_below(gg_draw(base, ctr++), (uint64_t)n);
        if (u == v) continue;
        const uint64_t a = u < v ? u : v, b = u < v ? v : u;
        if (!gg_set_insert(&set, gg_key(a, b))) continue;
        keys[2 * have] = gg_key(a, b);
        keys[2 * have + 1] = gg_key(b, a);
        ++have;
    }
    free(set.slot);
    return 2 * m;
}

/* ------------------------------------------------------------------ */
/* Planted dense block: k distinct ids drawn uniformly from [0, n) in   */
/* counter order (repeats rejected), written to `ids`; then each pair   */
/* (i < j) of the drawn list becomes an edge when its draw is below     */
/* p_fix (p scaled to 2^64, saturating).  Writes both directions;       */
/* returns the number of keys written (<= k(k-1)).                      */
/* ------------------------------------------------------------------ */
int64_t gg_planted_keys(int64_t n, int64_t k, uint64_t p_fix, uint64_t seed, uint64_t stream,
                        int32_t* ids, uint64_t* keys) {
    if (k < 0 || k > n || n > 0x7FFFFFFFLL) return -1;
    gg_set set;
    if (gg_set_init(&set, (uint64_t)k)) return -1;
    const uint64_t base = gg_base(seed, stream);
    uint64_t ctr = 0;
    int64_t have = 0;
    while (have < k) {
        const uint64_t v = gg_below(gg_draw(base, ctr++), (uint64_t)n);
        if (gg_set_insert(&set, v)) ids[have++] = (int32_t)v;
    }
    free(set.slot);
    const uint64_t pair_base = gg_base(seed, stream + 0x5151);
    int64_t out = 0;
    uint64_t pair = 0;
    for (int64_t i = 0; i < k; ++i) {
        for (int64_t j = i + 1; j < k; ++j, ++pair) {
            if (gg_draw(pair_base, pair) < p_fix) {
                keys[out++] = gg_key((uint64_t)ids[i], (uint64_t)ids[j]);
                keys[out++] = gg_key((uint64_t)ids[j], (uint64_t)ids[i]);
            }
        }
    }
    return out;
}

/* ------------------------------------------------------------------ */
/* Chung-Lu power law: weight w_i = (i+1)^(-1/(gamma-1)), endpoints of  */
/* each of `npairs` pairs drawn independently with probability          */
/* proportional to w (inverse CDF over the prefix sums).                */
/* Writes keys[2i], keys[2i+1]; loops become GG_NONE.                   */
/* ------------------------------------------------------------------ */
static int64_t chung_lu_core(int64_t n, int64_t npairs, double gamma, uint64_t seed,
                             uint64_t stream, uint64_t* keys, int parallel) {
    if (n < 1 || npairs < 0 || !(gamma > 1.0)) return -1;
    double* cdf = (double*)malloc((size_t)n * sizeof(double));
    if (!cdf) return -1;
    const double expo = -1.0 / (gamma - 1.0);
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        acc += pow((double)(i + 1), expo);
        cdf[i] = acc;
    }
    const double total = acc;
    const uint64_t base = gg_base(seed, stream);
#pragma omp parallel for schedule(static) if (parallel)
    for (int64_t p = 0; p < npairs; ++p) {
        uint64_t end[2];
        for (int e = 0; e < 2; ++e) {
            const uint64_t r = gg_draw(base, 2 * (uint64_t)p + (uint64_t)e);
            const double x = (double)(r >> 11) * (1.0 / 9007199254740992.0) * total;
            int64_t lo = 0, hi = n - 1; /* first i with cdf[i] > x */
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (cdf[mid] > x) hi = mid; else lo = mid + 1;
            }
            end[e] = (uint64_t)lo;
        }
        if (end[0] == end[1]) {
            keys[2 * p] = GG_NONE;
            keys[2 * p + 1] = GG_NONE;
        } else {
            keys[2 * p] = gg_key(end[0], end[1]);
            keys[2 * p + 1] = gg_key(end[1], end[0]);
        }
    }
    free(cdf);
    return 2 * npairs;
}

int64_t gg_chung_lu_keys(int64_t n, int64_t npairs, double gamma, uint64_t seed, uint64_t stream,
                         uint64_t* keys) {
    return chung_lu_core(n, npairs, gamma, seed, stream, keys, 1);
}

/* ------------------------------------------------------------------ */
/* Sort keys ascending and drop GG_NONE and repeats.  `tmp` must hold   */
/* `count` keys.  Result is in `keys`; returns the new count.           */
/* Parallel LSD radix sort, 8-bit digits, stable, skipping digits that  */
/* are constant over the input.                                         */
/* ------------------------------------------------------------------ */
int64_t gg_sort_unique(uint64_t* keys, uint64_t* tmp, int64_t count) {
    if (count <= 0) return 0;
    int nt = omp_get_max_threads();
    if (nt < 1) nt = 1;
    int64_t* cnt = (int64_t*)calloc((size_t)nt * 257, sizeof(int64_t));
    if (!cnt) return -1;

    /* 1. drop GG_NONE (stable compaction into tmp, then back) */
    {
        int64_t* part = (int64_t*)calloc((size_t)nt + 1, sizeof(int64_t));
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num();
            const int64_t lo = count * t / nt, hi = count * (t + 1) / nt;
            int64_t c = 0;
            for (int64_t i = lo; i < hi; ++i) c += keys[i] != GG_NONE;
            part[t + 1] = c;
#pragma omp barrier
#pragma omp single
            for (int i = 0; i < nt; ++i) part[i + 1] += part[i];
            int64_t o = part[t];
            for (int64_t i = lo; i < hi; ++i)
                if (keys[i] != GG_NONE) tmp[o++] = keys[i];
        }
        count = part[nt];
        free(part);
        memcpy(keys, tmp, (size_t)count * sizeof(uint64_t));
    }
    if (count == 0) { free(cnt); return 0; }

    /* 2. which digits vary */
    uint64_t orv = 0, andv = ~0ULL;
#pragma omp parallel for reduction(| : orv) reduction(& : andv) num_threads(nt)
    for (int64_t i = 0; i < count; ++i) { orv |= keys[i]; andv &= keys[i]; }
    const uint64_t vary = orv ^ andv;

    uint64_t* src = keys;
    uint64_t* dst = tmp;
    for (int d = 0; d < 8; ++d) {
        const int sh = 8 * d;
        if (((vary >> sh) & 0xFF) == 0) continue;
        memset(cnt, 0, (size_t)nt * 257 * sizeof(int64_t));
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num();
            const int64_t lo = count * t / nt, hi = count * (t + 1) / nt;
            int64_t* h = cnt + (size_t)t * 257;
            for (int64_t i = lo; i < hi; ++i) h[(src[i] >> sh) & 0xFF]++;
#pragma omp barrier
#pragma omp single
            {
                int64_t run = 0;
                for (int b = 0; b < 256; ++b)
                    for (int u = 0; u < nt; ++u) {
                        const int64_t c = cnt[(size_t)u * 257 + b];
                        cnt[(size_t)u * 257 + b] = run;
                        run += c;
                    }
            }
            for (int64_t i = lo; i < hi; ++i) {
                const uint64_t k = src[i];
                dst[h[(k >> sh) & 0xFF]++] = k;
            }
        }
        uint64_t* sw = src; src = dst; dst = sw;
    }
    if (src != keys) memcpy(keys, src, (size_t)count * sizeof(uint64_t));

    /* 3. unique (stable compaction of run heads) */
    {
        int64_t* part = (int64_t*)calloc((size_t)nt + 1, sizeof(int64_t));
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num();
            const int64_t lo = count * t / nt, hi = count * (t + 1) / nt;
            int64_t c = 0;
            for (int64_t i = lo; i < hi; ++i) c += (i == 0 || keys[i] != keys[i - 1]);
            part[t + 1] = c;
#pragma omp barrier
#pragma omp single
            for (int i = 0; i < nt; ++i) part[i + 1] += part[i];
            int64_t o = part[t];
            for (int64_t i = lo; i < hi; ++i)
                if (i == 0 || keys[i] != keys[i - 1]) tmp[o++] = keys[i];
        }
        count = part[nt];
        free(part);
        memcpy(keys, tmp, (size_t)count * sizeof(uint64_t));
    }
    free(cnt);
    return count;
}

/* ------------------------------------------------------------------ */
/* Sorted unique directed keys -> CSR.  row_ptr has n+1 entries.        */
/* Returns 0, or -1 if a key names a vertex >= n or the count exceeds   */
/* the int32 range.                                                     */
/* ------------------------------------------------------------------ */
int32_t gg_keys_to_csr(const uint64_t* keys, int64_t count, int64_t n, int32_t* row_ptr,
                       int32_t* col_idx) {
    if (n < 0 || count < 0 || count > 0x7FFFFFFFLL || n > 0x7FFFFFFELL) return -1;
    if (count > 0 && ((keys[count - 1] >> 32) >= (uint64_t)n)) return -1;
    int bad = 0;
#pragma omp parallel for reduction(| : bad)
    for (int64_t i = 0; i < count; ++i) {
        const uint64_t r = keys[i] >> 32, c = keys[i] & 0xFFFFFFFFULL;
        if (c >= (uint64_t)n) bad = 1;
        col_idx[i] = (int32_t)c;
        const int64_t prev = i == 0 ? -1 : (int64_t)(keys[i - 1] >> 32);
        for (int64_t q = prev + 1; q <= (int64_t)r; ++q) row_ptr[q] = (int32_t)i;
    }
    const int64_t last = count == 0 ? -1 : (int64_t)(keys[count - 1] >> 32);
    for (int64_t q = last + 1; q <= n; ++q) row_ptr[q] = (int32_t)count;
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Single-threaded sort + unique and CSR conversion, for building many  */
/* small graphs at once (one graph per OpenMP thread).                  */
/* ------------------------------------------------------------------ */
static int64_t sort_unique_serial(uint64_t* keys, uint64_t* tmp, int64_t count) {
    int64_t c = 0;
    for (int64_t i = 0; i < count; ++i)
        if (keys[i] != GG_NONE) keys[c++] = keys[i];
    count = c;
    if (count == 0) return 0;
    uint64_t orv = 0, andv = ~0ULL;
    for (int64_t i = 0; i < count; ++i) { orv |= keys[i]; andv &= keys[i]; }
    const uint64_t vary = orv ^ andv;
    uint64_t* src = keys;
    uint64_t* dst = tmp;
    int64_t cnt[257];
    for (int d = 0; d < 8; ++d) {
        const int sh = 8 * d;
        if (((vary >> sh) & 0xFF) == 0) continue;
        memset(cnt, 0, sizeof(cnt));
        for (int64_t i = 0; i < count; ++i) cnt[((src[i] >> sh) & 0xFF) + 1]++;
        for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
        for (int64_t i = 0; i < count; ++i) dst[cnt[(src[i] >> sh) & 0xFF]++] = src[i];
        uint64_t* sw = src; src = dst; dst = sw;
    }
    if (src != keys) memcpy(keys, src, (size_t)count * sizeof(uint64_t));
    c = 0;
    for (int64_t i = 0; i < count; ++i)
        if (i == 0 || keys[i] != keys[i - 1]) keys[c++] = keys[i];
    return c;
}

static int32_t keys_to_csr_serial(const uint64_t* keys, int64_t count, int64_t n,
                                  int32_t* row_ptr, int32_t* col_idx) {
    int64_t q = 0;
    for (int64_t i = 0; i < count; ++i) {
        const uint64_t r = keys[i] >> 32, c = keys[i] & 0xFFFFFFFFULL;
        if (r >= (uint64_t)n || c >= (uint64_t)n) return -1;
        while (q <= (int64_t)r) row_ptr[q++] = (int32_t)i;
        col_idx[i] = (int32_t)c;
    }
    while (q <= n) row_ptr[q++] = (int32_t)count;
    return 0;
}

/* ------------------------------------------------------------------ */
/* A batch of independent graphs.  Graph i is G(n_i, size_i) (kind 0,   */
/* Erdos-Renyi, same stream as gg_er_keys) or Chung-Lu with size_i      */
/* pairs and exponent gamma_i (kind 1, same stream as                   */
/* gg_chung_lu_keys), under seed_i, so it equals the graph the single   */
/* generators build from the same arguments.  Graphs are generated in   */
/* parallel, one per thread; gg_batch_copy then places them back to     */
/* back.                                                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n, count;
    int32_t* row_ptr;
    int32_t* col_idx;
} gg_one;

typedef struct {
    int32_t count;
    gg_one* g;
} gg_batch;

void gg_batch_free(void* h) {
    gg_batch* b = (gg_batch*)h;
    if (!b) return;
    for (int32_t i = 0; i < b->count; ++i) {
        free(b->g[i].row_ptr);
        free(b->g[i].col_idx);
    }
    free(b->g);
    free(b);
}

void* gg_batch_generate(int32_t count, const int32_t* kind, const int64_t* n, const int64_t* size,
                        const double* gamma, const uint64_t* seed, int64_t* m_out) {
    if (count < 0) return NULL;
    gg_batch* b = (gg_batch*)calloc(1, sizeof(gg_batch));
    if (!b) return NULL;
    b->count = count;
    b->g = (gg_one*)calloc((size_t)(count > 0 ? count : 1), sizeof(gg_one));
    if (!b->g) { free(b); return NULL; }
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
    for (int32_t i = 0; i < count; ++i) {
        const int64_t nk = 2 * size[i];
        uint64_t* keys = (uint64_t*)malloc((size_t)(nk > 0 ? nk : 1) * sizeof(uint64_t));
        uint64_t* tmp = (uint64_t*)malloc((size_t)(nk > 0 ? nk : 1) * sizeof(uint64_t));
        int64_t cnt = -1;
        if (keys && tmp) {
            if (kind[i] == 0)
                cnt = gg_er_keys(n[i], size[i], seed[i], 1, keys);
            else if (kind[i] == 1)
                cnt = chung_lu_core(n[i], size[i], gamma[i], seed[i], 4, keys, 0);
        }
        if (cnt >= 0) cnt = sort_unique_serial(keys, tmp, cnt);
        free(tmp);
        gg_one* o = &b->g[i];
        o->n = n[i];
        o->count = cnt;
        if (cnt < 0 || cnt > 0x7FFFFFFFLL || n[i] > 0x7FFFFFFELL) {
            fail = 1;
        } else {
            o->row_ptr = (int32_t*)malloc((size_t)(n[i] + 1) * sizeof(int32_t));
            o->col_idx = (int32_t*)malloc((size_t)(cnt > 0 ? cnt : 1) * sizeof(int32_t));
            if (!o->row_ptr || !o->col_idx ||
                keys_to_csr_serial(keys, cnt, n[i], o->row_ptr, o->col_idx) != 0)
                fail = 1;
            m_out[i] = cnt / 2;
        }
        free(keys);
    }
    if (fail) { gg_batch_free(b); return NULL; }
    return b;
}

int32_t gg_batch_copy(void* h, int32_t* row_ptr, int32_t* col_idx, const int64_t* rp_off,
                      const int64_t* ci_off) {
    gg_batch* b = (gg_batch*)h;
    if (!b) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t i = 0; i < b->count; ++i) {
        const gg_one* o = &b->g[i];
        memcpy(row_ptr + rp_off[i], o->row_ptr, (size_t)(o->n + 1) * sizeof(int32_t));
        if (o->count) memcpy(col_idx + ci_off[i], o->col_idx, (size_t)o->count * sizeof(int32_t));
    }
    return 0;
}
