// peel.hip - Bahmani's (2+2eps) peeling passes on gfx950 and the C ABI of
// libdsg.so (include/dsg.h).
//
// One pass of Algorithm 1 (P-Bahmani, Section 3.1) runs as seven kernels on
// the caller's stream:
//
//   k_mark_count    part 1, the failure test, over the live list L_{k-1}
//                   and its dense degree array: every vertex whose degree is
//                   <= T_k fails: removed_at = k, live bit cleared (pass 1
//                   writes removed_at and the live bits of every vertex).  Per tile of the live list it records the
//                   failures with degree > 0, the survivors, the CSR row
//                   length of the former and the degree sums of both groups.
//   k_scan_tiles    exclusive prefix of the tile records (one workgroup).
//   k_mark_scatter  compacts, in live-list order, the survivors (id and
//                   degree) into L_k and the failures with degree > 0 into
//                   the walk list.  It also writes the rank directory (per
//                   32-vertex word: live bits and the number of survivors
//                   before the word) and the start of every survivor-rank
//                   bin in the record buffer (prefix of survivor degrees).
//   k_walk          part 2, the neighbour walk.  The adjacency entries of the
//                   walk list form one flat range cut into equal tiles, so
//                   hub rows spread over many workgroups.  A neighbour still
//                   present gets its survivor rank from the rank directory,
//                   and a 16-bit record of it is appended to its rank bin;
//                   a tile reserves space once per bin it touches.  A
//                   neighbour outside the pass's survivor filter (few
//                   survivors) skips the rank-directory lookup.
//   k_walk_finish   one workgroup: sums the walk workgroups' record counts,
//                   reduces |V| and |E|, keeps the best graph, derives the
//                   next threshold and splits the bins into apply work items.
//   k_apply         the degree decrements.  Each work item counts its records
//                   in LDS (one counter per rank of the bin) and writes the
//                   counts as one partial row.
//   k_reduce        subtracts every bin's partial rows from the survivors'
//                   degrees (1 to 16 lanes per rank, by the rows per bin).
//
// A pass that leaves more survivors than the walk's survivor filter holds,
// and walks at least kIdMinEntries entries, keys its records by neighbour id
// instead (walk mode 2), so that no walked entry gathers from the rank
// directory:
//
//   k_walk_ids      takes the walk list in groups of kIdGroupTiles tiles and
//                   writes every walked entry as its neighbour's 16-bit
//                   position in a bucket of kIdWidth consecutive ids, the
//                   group's records sorted by bucket in LDS;
//   k_walk_finish   (phase 0) plans the apply items: one to a few per
//                   bucket, each over a range of record groups;
//   k_apply         counts a bucket's positions in LDS, finds the survivors
//                   among them from the bucket's rank-directory words and
//                   writes their counts as the item's partial row, indexed
//                   by position (workgroups take items from a counter);
//   k_reduce        sums each bucket's partial rows into its survivors'
//                   degrees;
//   k_walk_finish   (phase 1) completes the pass (|V|, |E|, best, threshold)
//                   from the counts that reached a survivor.
//
// The "barrier synchronization" between the two parts of Algorithm 1 is the
// kernel boundary between k_mark_scatter and k_walk.  The degree decrements
// of the paper's part 2 ("atomicSub" on the neighbour's degree) become
// binned LDS histograms: device-scope atomics on gfx950 sustain only a few
// tens of billions of operations per second, LDS atomics over a thousand.
//
// Exact integer arithmetic makes every result independent of launch shape
// and execution order.  The failure test deg * |V| * den <= 2(num+den)|E| is
// evaluated as deg <= T_k with T_k = floor(2(num+den)|E| / (|V| den)), the
// same test for integer deg.  Entries between two vertices that fail
// together are not counted one by one: a failed vertex of degree d has
// exactly d entries into the graph of the pass start, so intra = sum(d) -
// cross, and |E| drops by cross + intra / 2.  A survivor u receives at most
// deg(u) records in a pass, so the prefix of survivor degrees bounds every
// bin exactly.  Rows of vertices that fail with degree 0 are not walked, and
// nothing is walked in a pass that leaves no survivor.
//
// The live lists keep ascending id order (every compaction is stable and
// pass 1 starts from 0..n-1), so the survivors of pass k, as listed for
// pass k + 1, are S_k in the order the output wants: when pass k sets the
// best graph, pass k + 1's k_mark_count copies its live list to best_ids.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"
#include "dsg.h"
#include "host.h"

namespace dsg {

// Pointers into one workspace allocation.
struct Work {
    DevState* st;
    int32_t* removed_at;  // n: pass of failure, kNever while present
    uint2* dir;           // ceil(n/32): .x live bits, .y survivors before the word
    int32_t* list0;       // n: live lists, even passes
    int32_t* list1;       // n: live lists, odd passes
    int32_t* deg0;        // n: degrees aligned with list0
    int32_t* deg1;        // n: degrees aligned with list1
    int32_t* arow;        // n: walk list of the current pass (CSR row start of each vertex)
    int32_t* aoff;        // n+1: exclusive prefix of the walk list's row lengths
    int32_t* tile_first;  // walk tiles + 1: walk-list index owning each tile start
    int4* tiles;          // 2 per mark tile: counts, then their prefix
    int32_t* bin_start;   // bins + 1: record-buffer start of every rank bin
    int32_t* bin_cur;     // bins: append cursor of every rank bin
    int2* bin_items;      // bins: (first apply item, item count)
    int4* items;          // apply items: (bin, first record, end record, ranks)
    int32_t* partial;     // items x part_stride: per-item counts
    uint16_t* recs;       // walk tiles x kWalkTile: 16-bit local ranks
    uint16_t* toff;       // walk tiles x (bins + 1): bin offsets inside each tile (walk
                          // mode 2: buckets x record groups, 32-bit run bounds)
    uint32_t* filt;       // kFiltWords: survivor filter of the current pass
    unsigned long long* wpart;  // kMaxWalkGrid: decrement records per walk workgroup
    PassRecord* trace;    // kTraceCap
    int64_t* progress;    // pinned host word the tile scan posts to, or null
};

static_assert(sizeof(PassRecord) == sizeof(dsg_pass_trace), "trace layout");

__device__ inline const int32_t* live_in(const Work& w, int32_t pass) {
    return pass == 1 ? nullptr : ((pass - 1) & 1 ? w.list1 : w.list0);
}
__device__ inline int32_t* deg_in(const Work& w, int32_t pass) {
    return (pass - 1) & 1 ? w.deg1 : w.deg0;
}
__device__ inline int32_t* live_out(const Work& w, int32_t pass) {
    return (pass & 1) ? w.list1 : w.list0;
}
__device__ inline int32_t* deg_out(const Work& w, int32_t pass) {
    return (pass & 1) ? w.deg1 : w.deg0;
}

// out[j] = p[base + j] for base + j < lim, else `fill`; two 16-byte loads
// when the span is whole and 16-byte aligned.
__device__ inline void load8(const int32_t* __restrict__ p, int64_t base, int64_t lim,
                             int32_t fill, int32_t out[8]) {
    const int32_t* q = p + base;
    if (base + 8 <= lim && ((uintptr_t)q & 15u) == 0) {
        const int4 a = reinterpret_cast<const int4*>(q)[0];
        const int4 b = reinterpret_cast<const int4*>(q)[1];
        out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
        out[4] = b.x; out[5] = b.y; out[6] = b.z; out[7] = b.w;
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) out[j] = base + j < lim ? q[j] : fill;
    }
}

// p[base + j] = v[j] for base + j < lim; two 16-byte stores when the span is
// whole and 16-byte aligned.
__device__ inline void store8(int32_t* __restrict__ p, int64_t base, int64_t lim,
                              const int32_t v[8]) {
    int32_t* q = p + base;
    if (base + 8 <= lim && ((uintptr_t)q & 15u) == 0) {
        reinterpret_cast<int4*>(q)[0] = make_int4(v[0], v[1], v[2], v[3]);
        reinterpret_cast<int4*>(q)[1] = make_int4(v[4], v[5], v[6], v[7]);
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (base + j < lim) q[j] = v[j];
    }
}

// ------------------------------------------------------------------ init
// The state only: pass 1 reads every row offset (and flags a row_ptr that
// decreases anywhere before any later kernel uses one as an address) and
// writes every removal pass and every live-bit word.

__global__ void k_init_state(Work w, const int32_t* __restrict__ rp, int64_t n, int64_t m,
                             int64_t num, int64_t den, int32_t max_pass, int32_t trace_cap,
                             int32_t part_stride, int32_t max_items, int32_t force_bins,
                             int32_t id_mode, int32_t core_mode) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    DevState* st = w.st;
    st->S = n;
    st->E = m;
    st->best_E = m;
    st->best_S = n;
    st->eps_num = num;
    st->eps_den = den;
    st->nA = st->nL = st->edges = st->sumdeg = st->sumdeg_surv = 0;
    st->cross = 0;
    st->best_count = 0;
    st->tot_walked = st->tot_cross = st->tot_live = st->tot_alist = 0;
    st->chunk = 0;
    st->pass = 1;
    // core levels start at k = 0; the whole graph C_0 is the first candidate
    // and its cut (core number > cut) is -1
    st->T = core_mode ? 0 : pass_threshold(m, n, num, den);
    st->best_pass = core_mode ? -1 : 0;
    st->core_mode = core_mode;
    st->min_surv = INT32_MAX;
    st->jumped = 0;
    st->cb_nelig = st->cb_nlegit = 0;
    st->cb_sumlegit = st->cb_el = 0;
    st->done = 0;
    st->status = kStOk;
    st->max_pass = max_pass;
    st->trace_cap = trace_cap;
    st->n_tiles_walk = 0;
    st->nbins = 0;
    st->n_items = 0;
    st->part_stride = part_stride;
    st->max_items = max_items;
    st->walk_mode = 0;
    st->toff_stride = 1;
    st->force_bins = force_bins;
    st->apply_lanes = 64;
    st->reduce_lanes = 16;
    st->use_filt = 0;
    st->apply_direct = 0;
    st->id_mode = id_mode;
    st->id_nb = 0;
    st->id_groups = 0;
    st->id_words = 0;
    st->apply_next = 0;
    if (rp[0] != 0 || (int64_t)rp[n] != 2 * m) {
        st->status = kStBadRowPtr;
        st->done = 1;
    }
}

// ------------------------------------------------------------ mark: count

// `best` (may be null): S~ output.  S_k, the survivors of pass k, is this
// pass's live list, ascending; when pass k set the best graph the list is
// copied to `best` as it is loaded, so that after the last pass `best`
// holds S~ (S_0 = V, best pass 0, is written by k_extract_iota instead).
__global__ __launch_bounds__(kBlock) void k_mark_count(Work w, const int32_t* __restrict__ rp,
                                                       int64_t n, int32_t* __restrict__ best) {
    DevState* st = w.st;
    if (st->done) return;
    const int32_t pass = st->pass;
    const int64_t S = st->S;
    const int32_t T = st->T;
    const int32_t* __restrict__ lin = live_in(w, pass);
    const int32_t* __restrict__ din = deg_in(w, pass);
    const int64_t ntiles = (S + kMarkTile - 1) / kMarkTile;
    // what removed_at records: the pass, or in core mode the level (which is
    // the core number of every vertex removed at that level)
    const bool core = st->core_mode != 0;
    const int32_t rv = core ? T : pass;
    const bool copy_best = best && !core && lin && st->best_pass == pass - 1;
    if (copy_best && blockIdx.x == 0 && threadIdx.x == 0) st->best_count = S;
    __shared__ uint32_t red[5 * kWaves];

    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t base = t * kMarkTile + (int64_t)threadIdx.x * kMarkItems;
        // 1. loads: ids and degrees of this thread's entries
        static_assert(kMarkItems == 8, "8-wide loads");
        int32_t vv[kMarkItems], dd[kMarkItems];
        if (!lin) {
            int32_t r[kMarkItems];
            load8(rp, base, S + 1, 0, r);
            const int32_t r8 = base + 8 <= S ? rp[base + 8] : 0;
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) {
                vv[j] = base + j < S ? (int32_t)(base + j) : -1;
                dd[j] = (j + 1 < kMarkItems ? r[j + 1] : r8) - r[j];
            }
            // a row_ptr that decreases is no CSR: every later kernel sees
            // the run done (every writer stores the same values)
            bool bad = false;
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) bad |= vv[j] >= 0 && dd[j] < 0;
            if (bad) {
                st->status = kStBadRowPtr;
                st->done = 1;
            }
        } else {
            load8(lin, base, S, -1, vv);
            load8(din, base, S, 0, dd);
            if (copy_best) store8(best, base, S, vv);
        }
        int32_t ll[kMarkItems];
#pragma unroll
        for (int j = 0; j < kMarkItems; ++j)
            if ((uint64_t)(int64_t)vv[j] >= (uint64_t)n) vv[j] = -1;
        if (!lin) {
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) ll[j] = dd[j];
        } else {
            // row length of a failure with degree > 0, and in core mode of
            // every live vertex (pass 1: the degree itself); all row bounds
            // are loaded before any is used (row 0 stands in for the others)
            int32_t rs[kMarkItems], re[kMarkItems];
            bool need[kMarkItems];
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) {
                need[j] = vv[j] >= 0 && ((dd[j] <= T && dd[j] > 0) || core);
                const int32_t x = need[j] ? vv[j] : 0;
                rs[j] = rp[x];
                re[j] = rp[x + 1];
            }
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) ll[j] = need[j] ? re[j] - rs[j] : dd[j];
        }
        // 2. decisions, removal passes and live bits
        uint32_t cA = 0, cL = 0, cE = 0, cDr = 0, cDs = 0;
        uint32_t dmin = 0xFFFFFFFFu;  // least survivor degree
        uint32_t wi = 0xFFFFFFFFu, wm = 0;
        uint32_t gone8 = 0;  // pass 1: bit j set when entry j fails
#pragma unroll
        for (int j = 0; j < kMarkItems; ++j) {
            const int32_t v = vv[j];
            if (v < 0) continue;
            const int32_t d = dd[j];
            if (d <= T) {
                if (lin) {
                    w.removed_at[v] = rv;
                    const uint32_t word = (uint32_t)v >> 5;
                    if (word != wi) {
                        if (wm) atomicAnd(&w.dir[wi].x, ~wm);
                        wi = word;
                        wm = 0;
                    }
                    wm |= 1u << (v & 31);
                } else {
                    gone8 |= 1u << j;
                }
                cDr += (uint32_t)d;
                if (d > 0) {
                    ++cA;
                    cE += (uint32_t)ll[j];
                }
            } else {
                ++cL;
                cDs += (uint32_t)d;
                dmin = min(dmin, (uint32_t)d);
            }
        }
        if (lin) {
            if (wm) atomicAnd(&w.dir[wi].x, ~wm);
        } else {
            // pass 1: ids base..base+7 lie in one 32-vertex word that only the
            // four consecutive lanes (tid & ~3) .. (tid | 3) touch; they merge
            // their masks and one of them stores the word
            static_assert(kMarkItems == 8, "four lanes per 32-vertex word");
            if (base < S) {
                int32_t ra[kMarkItems];
#pragma unroll
                for (int j = 0; j < kMarkItems; ++j) ra[j] = (gone8 >> j & 1u) ? rv : kNever;
                store8(w.removed_at, base, S, ra);
            }
            uint32_t gone = gone8 << (8 * (threadIdx.x & 3));
            gone |= __shfl_xor(gone, 1, 64);
            gone |= __shfl_xor(gone, 2, 64);
            const int64_t wbase = base & ~(int64_t)31;
            if ((threadIdx.x & 3) == 0 && wbase < S) {
                const int64_t left = n - wbase;
                const uint32_t valid = left >= 32 ? 0xFFFFFFFFu : ((1u << left) - 1u);
                w.dir[wbase >> 5].x = valid & ~gone;
            }
        }
        // the five tile sums in one reduction; the least survivor degree
        // (core levels only) in a second one
        uint32_t sums[5] = {cA, cL, cE, cDr, cDs};
        block_sum_k<5>(sums, red);
        const uint32_t tMin = core ? block_min(dmin, red) : 0xFFFFFFFFu;
        // core levels: the survivors of least degree and their row lengths
        // (the failures of the next level if nothing fails at this one)
        uint32_t least[2] = {0u, 0u};
        if (core) {
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) {
                if (vv[j] >= 0 && dd[j] > T && (uint32_t)dd[j] == tMin) {
                    ++least[0];
                    least[1] += (uint32_t)ll[j];
                }
            }
            block_sum_k<2>(least, red);
        }
        if (threadIdx.x == 0) {
            w.tiles[2 * t] = make_int4((int)sums[0], (int)sums[1], (int)sums[2], (int)sums[3]);
            w.tiles[2 * t + 1] = make_int4((int)sums[4], (int)tMin, (int)least[0], (int)least[1]);
        }
    }
}

// ---------------------------------------------------- prefix of tile counts
// mode 0: the tiles of the current pass's live list (prefix of failures with
//         degree > 0, survivors, walk entries and survivor degrees; the
//         failures' degree sum is only totalled).
// mode 1: the extract tiles over 0..n-1 (component x).

// The records pass through LDS in chunks of up to kScanChunk tiles (132 KB),
// so that every global load and store covers consecutive records and a pass
// over 8192 tiles takes two round trips to memory.  Each thread sums a run
// of consecutive tiles: one tile while the tiles fit one per thread, up to
// kScanPer for more.  One 16-byte pad after every 32 records (a longest run)
// keeps the runs of eight neighbouring lanes in distinct banks.
constexpr int kScanPer = 16;
constexpr int kScanChunk = kScanBlock * kScanPer;
__device__ inline int scan_slot(int r) { return r + (r >> 5); }

// Posts 2 * seq + final to the host's progress word (system scope, so that
// the host sees it while the pass is still running): `seq` numbers the
// passes the host has enqueued, `final` says that no pass after this one
// has work, so the host enqueues no more.
// The progress word: 4 seq + 2 few + fin, where fin says that pass seq left
// no survivor (or that the peel had ended) and few that it left at most
// kFiltBits survivors, so that no later pass can key its records by
// neighbour id unless a launch flag forces it.
__device__ inline void post_progress(int64_t* p, int64_t seq, bool fin, bool few) {
    __hip_atomic_store(p, 4 * seq + (few ? 2 : 0) + (fin ? 1 : 0), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(Work w, int32_t mode, int64_t n,
                                                           int64_t seq) {
    static_assert(kScanBlock == kBlock, "the block reductions assume kWaves waves");
    DevState* st = w.st;
    if (mode == 0) {
        if (st->done) {
            if (threadIdx.x == 0 && w.progress) post_progress(w.progress, seq, true, true);
            return;
        }
    } else {
        if (!st->done || st->status != kStOk) return;
    }
    const int64_t items = mode == 0 ? st->S : n;
    const int64_t nt = (items + kMarkTile - 1) / kMarkTile;
    const int tid = threadIdx.x;
    __shared__ int4 buf[2 * kScanChunk + 2 * kScanChunk / 32];
    __shared__ uint32_t red[5 * kWaves];

    // Core levels: when nothing fails at level T, the level has ended.  The
    // next level is the least degree left, and the vertices failing there
    // are exactly those of that degree, which every tile has counted (with
    // their row lengths); the pass becomes the next level's first pass.
    bool jump = false;
    uint32_t jmin = 0xFFFFFFFFu;
    if (mode == 0 && st->core_mode) {
        uint32_t l0[1] = {0u};  // survivors (< 2^31)
        uint32_t mn0 = 0xFFFFFFFFu;
        for (int64_t i = tid; i < nt; i += kScanBlock) {
            l0[0] += (uint32_t)w.tiles[2 * i].y;
            mn0 = min(mn0, (uint32_t)w.tiles[2 * i + 1].y);
        }
        block_sum_k<1>(l0, red);
        jmin = block_min(mn0, red);
        jump = items > 0 && (int64_t)l0[0] == items;
    }
    // running totals of the chunks before; every partial sum below is a
    // count of vertices or of adjacency entries, so it fits 32 bits
    int64_t ca = 0, cl = 0, ce = 0, cds = 0, cdr = 0;
    uint32_t mn = 0xFFFFFFFFu;
    const int per = (int)std::min<int64_t>(
        kScanPer, std::max<int64_t>(1, (nt + kScanBlock - 1) / kScanBlock));
    const int chunk = per * kScanBlock;
    for (int64_t c0 = 0; c0 < nt; c0 += chunk) {
        const int cn = (int)std::min<int64_t>(chunk, nt - c0);
        const int4* __restrict__ src = w.tiles + 2 * c0;
#pragma unroll 8
        for (int r = tid; r < 2 * cn; r += kScanBlock) buf[scan_slot(r)] = src[r];
        __syncthreads();
        // this thread's run: failures with degree > 0, survivors, walk
        // entries, survivor degrees and failure degrees
        uint32_t v[5] = {0u, 0u, 0u, 0u, 0u};
        const int i0 = tid * per;
#pragma unroll 4
        for (int k = 0; k < per; ++k) {
            const int i = i0 + k;
            if (i < cn) {
                const int4 c = buf[scan_slot(2 * i)];
                const int4 q = buf[scan_slot(2 * i + 1)];
                if (!jump) {
                    v[0] += (uint32_t)c.x;
                    v[1] += (uint32_t)c.y;
                    v[2] += (uint32_t)c.z;
                    v[4] += (uint32_t)c.w;
                    if (mode == 0) {
                        v[3] += (uint32_t)q.x;
                        mn = min(mn, (uint32_t)q.y);
                    }
                } else {
                    // the next level's failures: the least-degree vertices of
                    // the tiles whose least degree is the global one
                    const uint32_t kk = (uint32_t)q.y == jmin ? (uint32_t)q.z : 0u;
                    v[0] += kk;
                    v[1] += (uint32_t)c.y - kk;
                    v[2] += kk ? (uint32_t)q.w : 0u;
                    v[4] += kk * jmin;
                    v[3] += (uint32_t)q.x - kk * jmin;
                }
            }
        }
        uint32_t tot[5];
        block_excl_sum_k<5>(v, red, tot);
        int64_t pa = ca + v[0], pl = cl + v[1], pe = ce + v[2], pds = cds + v[3];
#pragma unroll 4
        for (int k = 0; k < per; ++k) {
            const int i = i0 + k;
            if (i < cn) {
                const int4 c = buf[scan_slot(2 * i)];
                const int4 q = buf[scan_slot(2 * i + 1)];
                buf[scan_slot(2 * i)] = make_int4((int)pa, (int)pl, (int)pe, c.w);
                buf[scan_slot(2 * i + 1)] = make_int4((int)pds, 0, 0, 0);
                if (!jump) {
                    pa += (uint32_t)c.x;
                    pl += (uint32_t)c.y;
                    pe += (uint32_t)c.z;
                    if (mode == 0) pds += (uint32_t)q.x;
                } else {
                    const int64_t kk = (uint32_t)q.y == jmin ? q.z : 0;
                    pa += kk;
                    pl += c.y - kk;
                    pe += kk ? (uint32_t)q.w : 0u;
                    pds += (uint32_t)q.x - kk * (int64_t)jmin;
                }
            }
        }
        __syncthreads();
        int4* __restrict__ dst = w.tiles + 2 * c0;
#pragma unroll 8
        for (int r = tid; r < 2 * cn; r += kScanBlock) dst[r] = buf[scan_slot(r)];
        __syncthreads();  // the next chunk reuses buf
        ca += tot[0];
        cl += tot[1];
        ce += tot[2];
        cds += tot[3];
        cdr += tot[4];
    }
    const uint32_t tmin = block_min(mn, red);
    const int64_t ta = ca, tl = cl, te = ce, tds = cds, tdr = cdr;
    // few survivors: k_mark_scatter sets their bits in a cleared filter
    const bool filt = mode == 0 && tl > 0 && tl <= kFiltBits;
    if (filt)
        for (int i = threadIdx.x; i < kFiltWords; i += kScanBlock) w.filt[i] = 0u;
    if (threadIdx.x == 0) {
        if (mode == 0) {
            if (jump) {
                // what is left is the (T+1)-core: compare it with the best
                // (strict), as at the end of every level; the cut below its
                // core numbers is T
                if (st->E * st->best_S > st->best_E * st->S) {
                    st->best_E = st->E;
                    st->best_S = st->S;
                    st->best_pass = st->T;
                }
                st->T = (int32_t)jmin;
            }
            st->jumped = jump ? 1 : 0;
            st->nA = ta;
            st->nL = tl;
            st->edges = te;
            st->sumdeg = tdr;
            st->sumdeg_surv = tds;
            // the least survivor degree matters only after a pass that
            // removed nothing, which a jumped pass never is
            st->min_surv = (int32_t)min(tmin, (uint32_t)INT32_MAX);
            st->n_tiles_walk = (int32_t)((te + kWalkTile - 1) / kWalkTile);
            st->nbins = (int32_t)((tl + kBinWidth - 1) >> kBinShift);
            // Neighbour-id buckets when the survivor filter is off (more
            // survivors than it holds) and the walk is long: there every
            // walked entry would otherwise gather its neighbour's
            // rank-directory word, and the saving repays the id-keyed pass's
            // fixed costs (its apply items and two more launches; measured
            // to break even near 2^25 entries).  Not for core levels (light
            // passes) or forced bin regions.
            const int64_t nb2 = (n + kIdWidth - 1) >> kIdShift;
            const bool ids = !st->core_mode && !st->force_bins && st->id_mode != 2 && tl > 0 &&
                             te > 0 && nb2 <= kIdMaxBuckets &&
                             (st->id_mode == 1 || (tl > kFiltBits && te >= kIdMinEntries));
            st->walk_mode = ids ? 2 : (st->nbins <= kNbLds && !st->force_bins) ? 0 : 1;
            st->id_nb = (int32_t)nb2;
            st->id_groups = (int32_t)((te + kIdGroup - 1) / kIdGroup);
            st->id_words = (int32_t)((n + 31) >> 5);
            st->toff_stride = st->nbins + 1;
            st->use_filt = filt ? 1 : 0;
            st->tot_live += items;
            st->tot_alist += ta;
            st->cross = 0;
            w.aoff[ta] = (int32_t)te;
            w.bin_start[st->nbins] = (int32_t)tds;
            // a pass that leaves no survivor ends the run
            if (w.progress) post_progress(w.progress, seq, tl == 0, tl <= kFiltBits);
        } else {
            st->best_count = ta;
        }
    }
}

// ---------------------------------------------------------- mark: scatter

__global__ __launch_bounds__(kBlock) void k_mark_scatter(Work w, const int32_t* __restrict__ rp,
                                                         int64_t n, int64_t walk_cap,
                                                         int64_t bin_cap) {
    const DevState* st = w.st;
    if (st->done) return;
    const int32_t pass = st->pass;
    const int64_t S = st->S;
    const int32_t T = st->T;
    const int32_t* __restrict__ lin = live_in(w, pass);
    const int32_t* __restrict__ din = deg_in(w, pass);
    int32_t* __restrict__ lout = live_out(w, pass);
    int32_t* __restrict__ dout = deg_out(w, pass);
    const bool filt = st->use_filt != 0;
    // a pass the tile scan moved to the next core level: k_mark_count saw no
    // failure, so the removal level and the live bits are written here
    const bool jumped = st->jumped != 0;
    // a pass that leaves no survivor walks nothing: no walk tiles to mark
    const int64_t wcap = st->nL > 0 ? walk_cap : 0;
    const int64_t ntiles = (S + kMarkTile - 1) / kMarkTile;
    __shared__ uint32_t red[3 * kWaves];
    // the tile's walk-list rows (row start, prefix), staged so that they are
    // stored as consecutive runs
    __shared__ int32_t s_row[kMarkTile], s_off[kMarkTile];

    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t base = t * kMarkTile + (int64_t)threadIdx.x * kMarkItems;
        // the tile's prefix record and the element before this thread's
        // first one are loaded with the data, not after the block scan
        const int4 tp = w.tiles[2 * t];
        const int4 tq = w.tiles[2 * t + 1];
        int32_t prev = -1;
        if (base > 0 && base - 1 < S) prev = lin ? lin[base - 1] : (int32_t)(base - 1);
        int32_t vv[kMarkItems];
        int32_t dd[kMarkItems];
        int32_t ll[kMarkItems];
        int32_t rs[kMarkItems];  // CSR row start of every entry
        if (!lin) {
            int32_t r[kMarkItems];
            load8(rp, base, S + 1, 0, r);
            const int32_t r8 = base + 8 <= S ? rp[base + 8] : 0;
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) {
                vv[j] = base + j < S ? (int32_t)(base + j) : -1;
                dd[j] = (j + 1 < kMarkItems ? r[j + 1] : r8) - r[j];
                rs[j] = r[j];
                ll[j] = dd[j];
            }
        } else {
            load8(lin, base, S, -1, vv);
            load8(din, base, S, 0, dd);
            // row bounds of the failures with degree > 0, all loaded before
            // any is used (row 0 stands in for the other entries)
            int32_t re[kMarkItems];
            bool need[kMarkItems];
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) {
                need[j] = (uint64_t)(int64_t)vv[j] < (uint64_t)n && dd[j] <= T && dd[j] > 0;
                const int32_t x = need[j] ? vv[j] : 0;
                rs[j] = rp[x];
                re[j] = rp[x + 1];
            }
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) {
                ll[j] = need[j] ? re[j] - rs[j] : 0;
                if (!need[j]) rs[j] = 0;
            }
        }
        uint32_t cA = 0, cL = 0, cE = 0, cDs = 0;
#pragma unroll
        for (int j = 0; j < kMarkItems; ++j) {
            if ((uint64_t)(int64_t)vv[j] >= (uint64_t)n) {
                vv[j] = -1;
                continue;
            }
            if (dd[j] <= T) {
                if (dd[j] > 0) {
                    ++cA;
                    cE += (uint32_t)ll[j];
                }
            } else {
                ++cL;
                cDs += (uint32_t)dd[j];
            }
        }
        // the element before this thread's first one (prev) decides word
        // leadership
        uint32_t ex[3] = {cA | (cL << 16), cE, cDs}, tot[3];
        block_excl_sum_k<3>(ex, red, tot);
        const uint32_t ex_packed = ex[0], ex_e = ex[1], ex_ds = ex[2];
        const int64_t a0 = tp.x;  // the tile's first walk-list slot
        const int32_t tot_a = (int32_t)(tot[0] & 0xFFFFu);
        int64_t pA = a0 + (ex_packed & 0xFFFFu);
        int64_t pL = (int64_t)tp.y + (ex_packed >> 16);
        int64_t pE = (int64_t)(uint32_t)tp.z + ex_e;
        int64_t pD = (int64_t)(uint32_t)tq.x + ex_ds;
#pragma unroll
        for (int j = 0; j < kMarkItems; ++j) {
            const int32_t v = vv[j];
            if (v < 0) continue;
            if (prev < 0 || (prev >> 5) != (v >> 5)) w.dir[v >> 5].y = (uint32_t)pL;
            prev = v;
            if (dd[j] <= T) {
                if (jumped) {
                    w.removed_at[v] = T;
                    atomicAnd(&w.dir[v >> 5].x, ~(1u << (v & 31)));
                }
                if (dd[j] > 0 && pA < n) {
                    s_row[pA - a0] = rs[j];
                    s_off[pA - a0] = (int32_t)pE;
                    const int64_t len = ll[j];
                    // walk tiles whose first entry lies in [pE, pE + len)
                    for (int64_t tt = (pE + kWalkTile - 1) / kWalkTile;
                         tt * kWalkTile < pE + len && tt < wcap; ++tt)
                        w.tile_first[tt] = (int32_t)pA;
                    ++pA;
                    pE += len;
                }
            } else if (pL < n) {
                lout[pL] = v;
                dout[pL] = dd[j];
                if (filt) {
                    const uint32_t h = filt_hash((uint32_t)v);
                    atomicOr(&w.filt[h >> 5], 1u << (h & 31));
                }
                if ((pL & (kBinWidth - 1)) == 0 && (pL >> kBinShift) < bin_cap) {
                    w.bin_start[pL >> kBinShift] = (int32_t)pD;
                    w.bin_cur[pL >> kBinShift] = (int32_t)pD;
                }
                ++pL;
                pD += dd[j];
            }
        }
        // (the next tile writes s_row only after the barriers of its scan)
        __syncthreads();
        for (int i = threadIdx.x; i < tot_a && a0 + i < n; i += kBlock) {
            w.arow[a0 + i] = s_row[i];
            w.aoff[a0 + i] = s_off[i];
        }
    }
}

// --------------------------------------------------------- pass completion
// Run by every thread of k_walk_finish's workgroup.

__device__ void finish_pass(const Work& w, int32_t* s_flag, int32_t* red) {
    DevState* st = w.st;
    if (threadIdx.x == 0) {
        int32_t keep = 1;
        const int64_t cross = (int64_t)st->cross;
        const int64_t S_in = st->S, E_in = st->E;
        const int64_t S_out = st->nL;
        const int64_t intra = st->sumdeg - cross;
        const int32_t pass = st->pass;
        const int64_t E_out = E_in - cross - intra / 2;
        if (st->status != kStOk || intra < 0 || (intra & 1) || E_out < 0 ||
            (S_out == 0 && E_out != 0)) {
            if (st->status == kStOk) st->status = kStInvariant;
            st->done = 1;
            keep = 0;
        } else {
            if (pass <= st->trace_cap) {
                PassRecord r;
                r.s_in = S_in;
                r.e_in = E_in;
                r.thresh = st->T;
                r.removed = S_in - S_out;
                r.cross = cross;
                r.intra = intra;
                r.walked = S_out > 0 ? st->edges : 0;
                r.s_out = S_out;
                r.e_out = E_out;
                w.trace[pass - 1] = r;
            }
            st->tot_walked += S_out > 0 ? st->edges : 0;
            st->tot_cross += cross;
            // the best candidate: after every pass, or in core mode after a
            // pass that removed nothing (the level is done and what is left
            // is the (T+1)-core; best_pass then holds T, the cut below the
            // core numbers of the kept vertices)
            const bool level_end = S_out == S_in;
            const bool candidate = st->core_mode ? level_end : true;
            if (candidate && S_out > 0 && E_out * st->best_S > st->best_E * S_out) {
                st->best_E = E_out;
                st->best_S = S_out;
                st->best_pass = st->core_mode ? st->T : pass;
            }
            st->S = S_out;
            st->E = E_out;
            if (S_out == 0) {
                st->done = 1;
                keep = 0;
            } else if (pass + 1 > st->max_pass) {
                st->status = kStWatchdog;
                st->done = 1;
                keep = 0;
            } else {
                if (!st->core_mode)
                    st->T = pass_threshold(E_out, S_out, st->eps_num, st->eps_den);
                else if (level_end)
                    st->T = st->min_surv;  // the next non-empty level
                st->pass = pass + 1;
                st->chunk = std::max<int64_t>(kChunkMin, (cross + kTargetItems - 1) / kTargetItems);
            }
        }
        *s_flag = keep;
    }
    __syncthreads();
    // walk mode 2 completes the pass after its degree update
    if (st->walk_mode == 2) return;
    // no records (a pass that removed nothing, or whose failures had no
    // surviving neighbour): every partial count would be zero, so the apply
    // kernels have nothing to do
    if (!*s_flag || st->cross == 0) {
        if (threadIdx.x == 0) {
            st->n_items = 0;
            st->apply_direct = 0;
        }
        return;
    }
    const int32_t nb = st->nbins;
    const int64_t nL = st->nL;
    if (st->walk_mode == 0) {
        // records sit in per-tile regions: an item is one bin over a range of
        // tiles; a bin's items are consecutive
        const int32_t cap_a = st->max_items;
        const int64_t ntiles = st->n_tiles_walk;
        // items per bin: with one or two bins, half as many items (fewer
        // partial rows to write and reduce) measured faster; with more bins,
        // the full count keeps every CU busy
        const int64_t target = nb <= 2 ? kTargetItems / 2 : kTargetItems;
        const int64_t ipb = std::max<int64_t>(1, std::min<int64_t>(ntiles, target / nb));
        const int64_t tpi = (ntiles + ipb - 1) / ipb;
        const int64_t total_a = (int64_t)nb * ipb;
        for (int64_t i = threadIdx.x; i < total_a && i < cap_a; i += kBlock) {
            const int32_t b = (int32_t)(i / ipb);
            const int64_t t0 = std::min<int64_t>(ntiles, (i % ipb) * tpi);
            const int64_t t1 = std::min<int64_t>(ntiles, t0 + tpi);
            const int32_t ranks =
                (int32_t)std::min<int64_t>(kBinWidth, nL - ((int64_t)b << kBinShift));
            w.items[i] = make_int4(b, (int)t0, (int)t1, ranks);
        }
        for (int32_t b = threadIdx.x; b < nb; b += kBlock)
            w.bin_items[b] = make_int2((int)(b * ipb), total_a <= cap_a ? (int)ipb : 0);
        if (threadIdx.x == 0) {
            // lanes per (tile, bin) run in k_apply: about four batches of
            // loads per lane cover a mean run, so a wave counts several runs
            // at once (at least 8 lanes per run)
            const int64_t runs = std::max<int64_t>(1, ntiles * nb);
            const int64_t mean = (int64_t)st->cross / runs;
            int32_t lanes = 8;
            while (lanes < 64 && kApplyBatch * lanes * 4 < mean) lanes *= 2;
            st->apply_lanes = lanes;
            // lanes per rank in k_reduce: about four partial rows per lane
            int32_t rl = 1;
            while (rl < 16 && 4 * rl < ipb) rl *= 2;
            st->reduce_lanes = rl;
            if (total_a > cap_a) {  // cannot happen: nb * ipb <= max(nb, kTargetItems)
                st->status = kStInvariant;
                st->done = 1;
                st->n_items = 0;
            } else {
                st->n_items = (int32_t)total_a;
            }
            // few records (light k-core levels, the last passes of a peel):
            // partial rows and their reduction would cost the whole
            // survivor range, the nonzero counts at most a few thousand
            // device atomics (one per rank and item, however many records
            // a hub receives)
            st->apply_direct = (int64_t)st->cross <= kDirectRecords ? 1 : 0;
        }
        return;
    }
    // records sit in bin regions: split every bin into items of <= chunk records
    if (threadIdx.x == 0) {
        st->reduce_lanes = 16;
        st->apply_direct = 0;
    }
    const int64_t ch = st->chunk;
    const int32_t per = (nb + kBlock - 1) / kBlock;
    const int32_t lo = std::min<int32_t>(nb, per * (int32_t)threadIdx.x);
    const int32_t hi = std::min<int32_t>(nb, lo + per);
    int32_t cnt = 0;
    for (int32_t b = lo; b < hi; ++b) {
        const int64_t fill = (int64_t)__hip_atomic_load(&w.bin_cur[b], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT) -
                             w.bin_start[b];
        cnt += (int32_t)((fill + ch - 1) / ch);
    }
    int32_t total;
    int32_t first = block_excl_sum(cnt, red, &total);
    const int32_t cap = st->max_items;
    for (int32_t b = lo; b < hi; ++b) {
        const int64_t s0 = w.bin_start[b];
        const int64_t fill = (int64_t)__hip_atomic_load(&w.bin_cur[b], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT) - s0;
        const int32_t k = (int32_t)((fill + ch - 1) / ch);
        const int32_t ranks = (int32_t)std::min<int64_t>(kBinWidth, nL - ((int64_t)b << kBinShift));
        w.bin_items[b] = make_int2(first, first + k <= cap ? k : 0);
        for (int32_t j = 0; j < k && first + j < cap; ++j) {
            const int64_t a = s0 + (int64_t)j * ch;
            const int64_t z = std::min<int64_t>(s0 + fill, a + ch);
            w.items[first + j] = make_int4(b, (int)a, (int)z, ranks);
        }
        first += k;
    }
    if (threadIdx.x == 0) {
        if (total > cap) {  // cannot happen: the chunk size bounds the item count
            st->status = kStInvariant;
            st->done = 1;
            st->n_items = 0;
        } else {
            st->n_items = total;
        }
    }
}

// ------------------------------------------------------------------ walk
// All positions are 32-bit: 2m <= INT32_MAX, so every adjacency position,
// walk offset and tile start fits.

// popcount of `mask` over the lanes below this one
__device__ inline int32_t lanes_below(unsigned long long mask) {
    return (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Row base (CSR row start minus walk offset) of this thread's entries
// j * kBlock + tid of the walk tile that starts at entry e0 and spans the
// walk-list rows i0 .. i0 + c - 1.  A tile inside at most kFewRows rows
// compares each position with the row starts (the same values in every
// lane); a longer span builds an owner table in LDS: rows start at strictly
// increasing offsets, so a running max over the start marks works (indices
// < kWalkTile + 1 fit 16 bits; 8 per 16-byte word).  `clear` runs before the
// table's first barrier, and in the short case before one barrier when
// `sync_few` is set; the caller synchronises before own[] and bas[] are
// written again.
template <typename Clear>
__device__ __forceinline__ void tile_row_bases(const Work& w, int32_t i0, int32_t c, uint32_t e0,
                                               int32_t len, int32_t (&rb)[kWalkItems],
                                               uint16_t* own, int32_t* bas, int32_t* red,
                                               bool sync_few, Clear clear) {
    const int tid = threadIdx.x;
    const int32_t* __restrict__ aoff = w.aoff;
    const int32_t* __restrict__ arow = w.arow;
    if (c <= kFewRows) {
        int32_t fo[kFewRows], fb[kFewRows];
#pragma unroll
        for (int r = 0; r < kFewRows; ++r) {
            // rows past the span repeat the last one, which selects the same
            const int32_t i = i0 + min(r, c - 1);
            const int32_t ao = aoff[i];
            fo[r] = ao - (int32_t)e0;
            fb[r] = arow[i] - ao;
        }
#pragma unroll
        for (int j = 0; j < kWalkItems; ++j) {
            const int32_t p = min(j * kBlock + tid, len - 1);
            int32_t b = fb[0];
#pragma unroll
            for (int r = 1; r < kFewRows; ++r) b = fo[r] <= p ? fb[r] : b;
            rb[j] = b;
        }
        if (sync_few) {
            clear();
            __syncthreads();
        }
    } else {
        constexpr int kQ = kWalkItems / 8;  // 16-byte words of own[] per thread
        uint4* own4 = reinterpret_cast<uint4*>(own);
#pragma unroll
        for (int q = 0; q < kQ; ++q) own4[kQ * tid + q] = make_uint4(0u, 0u, 0u, 0u);
        clear();
        __syncthreads();
        // rows in rounds of four per thread, every load of a round issued
        // before any is used (indices clamped to the last row)
        for (int32_t r0 = 0; r0 < c; r0 += 4 * kBlock) {
            int32_t ao[4], ar[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t i = min(r0 + q * kBlock + tid, c - 1);
                ao[q] = aoff[i0 + i];
                ar[q] = arow[i0 + i];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t i = r0 + q * kBlock + tid;
                if (i < c) {
                    bas[i] = ar[q] - ao[q];
                    const int32_t o = ao[q] - (int32_t)e0;
                    if (o < len) own[o > 0 ? o : 0] = (uint16_t)i;
                }
            }
        }
        __syncthreads();
        {
            uint4 q4[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) q4[q] = own4[kQ * tid + q];
            uint32_t run = 0;
            auto step = [&run](uint32_t x) {
                const uint32_t lo = run = max(run, x & 0xFFFFu);
                const uint32_t hi = run = max(run, x >> 16);
                return lo | (hi << 16);
            };
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                q4[q].x = step(q4[q].x);
                q4[q].y = step(q4[q].y);
                q4[q].z = step(q4[q].z);
                q4[q].w = step(q4[q].w);
            }
            const uint32_t carry = (uint32_t)block_excl_max((int32_t)run, red, 0);
            auto lift = [carry](uint32_t x) {
                return max(x & 0xFFFFu, carry) | (max(x >> 16, carry) << 16);
            };
#pragma unroll
            for (int q = 0; q < kQ; ++q)
                own4[kQ * tid + q] = make_uint4(lift(q4[q].x), lift(q4[q].y), lift(q4[q].z),
                                                lift(q4[q].w));
        }
        __syncthreads();

#pragma unroll
        for (int j = 0; j < kWalkItems; ++j) rb[j] = own[min(j * kBlock + tid, len - 1)];
#pragma unroll
        for (int j = 0; j < kWalkItems; ++j) rb[j] = bas[rb[j]];
    }
}

__global__ __launch_bounds__(kBlock) void k_walk(Work w, const int32_t* __restrict__ ci,
                                                 uint32_t n, uint32_t nnz) {
    DevState* st = w.st;
    if (st->done || st->walk_mode == 2) return;
    const int32_t nA = (int32_t)st->nA;
    const uint32_t total = (uint32_t)st->edges;
    // no survivor: no decrement is possible and the rows need no walk
    const int32_t ntiles = st->nL > 0 ? st->n_tiles_walk : 0;
    const int32_t nb = st->nbins;
    const bool lds_bins = st->walk_mode == 0;
    const bool one_bin = nb == 1;
    const uint2* __restrict__ dir = w.dir;
    int32_t* __restrict__ bin_cur = w.bin_cur;
    uint16_t* __restrict__ recs = w.recs;
    const int tid = threadIdx.x;
    const bool filt = st->use_filt != 0;

    __shared__ __align__(16) uint16_t own[kWalkTile];
    __shared__ int32_t bas[kWalkTile + 1];
    __shared__ __align__(16) uint32_t filt_s[kFiltWords];
    __shared__ int32_t tcount[kNbLds];  // per-tile bin counts, then their offsets
    __shared__ int32_t wtot[kWaves];  // per-wave record counts (one bin)
    __shared__ int32_t red[kWaves];
    __shared__ unsigned long long redc[kWaves];

    if (filt && (int32_t)blockIdx.x < ntiles) {
        // read before the first tile's barriers
        const uint4* __restrict__ src = reinterpret_cast<const uint4*>(w.filt);
        uint4* dst = reinterpret_cast<uint4*>(filt_s);
        for (int i = tid; i < kFiltWords / 4; i += kBlock) dst[i] = src[i];
    }

    uint32_t cross = 0;
    // the walk-list rows that own a tile's first entry and the next tile's
    // (nA - 1 past the last tile), loaded one tile ahead
    auto row_of = [&](int32_t t) { return t < ntiles ? w.tile_first[t] : nA - 1; };
    int32_t i0_next = 0, ihi_next = 0;
    if ((int32_t)blockIdx.x < ntiles) {
        i0_next = row_of(blockIdx.x);
        ihi_next = row_of(blockIdx.x + 1);
    }
    for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t e0 = (uint32_t)t * kWalkTile;
        const int32_t len = (int32_t)min((uint32_t)kWalkTile, total - e0);
        const int32_t i0 = i0_next, ihi = ihi_next;
        if (t + (int32_t)gridDim.x < ntiles) {
            i0_next = row_of(t + gridDim.x);
            ihi_next = row_of(t + gridDim.x + 1);
        }
        if (i0 < 0 || ihi >= nA || ihi < i0 || ihi - i0 + 1 > kWalkTile + 1) {
            // cannot happen for a consistent walk list; never index with it
            if (tid == 0) st->status = kStInvariant;
            continue;
        }
        const int32_t c = ihi - i0 + 1;

        // 1. row base (CSR row start minus walk offset) of every entry
        int32_t rb[kWalkItems];
        tile_row_bases(w, i0, c, e0, len, rb, own, bas, red, lds_bins && !one_bin, [&] {
            if (lds_bins)
                for (int b = tid; b < nb; b += kBlock) tcount[b] = 0;
        });

        // 2. neighbour ids (coalesced: consecutive lanes, consecutive
        //    entries), all loads issued before any is used, with clamped
        //    indices and no load inside a branch (lanes past the tile end
        //    re-read its last entry); validity is applied after the last load.
        int32_t u[kWalkItems];
#pragma unroll
        for (int j = 0; j < kWalkItems; ++j) {
            const uint32_t p = (uint32_t)min(j * kBlock + tid, len - 1);
            const uint32_t pos = min((uint32_t)rb[j] + e0 + p, nnz - 1u);
            u[j] = __builtin_nontemporal_load(ci + pos);
        }
#pragma unroll
        for (int j = 0; j < kWalkItems; ++j)  // ids outside 0..n-1 are ignored
            if (j * kBlock + tid >= len || (uint32_t)u[j] >= n) u[j] = -1;
        // 3. survivor rank of every neighbour still present, else -1.  A
        //    neighbour outside the survivor filter gathers word 0 instead (one
        //    line for the whole wave) and is known not to survive.
        bool cand[kWalkItems];
#pragma unroll
        for (int j = 0; j < kWalkItems; ++j) cand[j] = u[j] >= 0;
        if (filt) {
#pragma unroll
            for (int j = 0; j < kWalkItems; ++j) {
                const uint32_t h = filt_hash((uint32_t)u[j]);
                cand[j] = cand[j] && ((filt_s[h >> 5] >> (h & 31)) & 1u);
            }
        }
        int32_t rk[kWalkItems];
#pragma unroll
        for (int j = 0; j < kWalkItems; ++j) {
            const uint32_t x = cand[j] ? (uint32_t)u[j] : 0u;
            const uint2 d = dir[x >> 5];
            const uint32_t bit = 1u << (x & 31);
            rk[j] = (cand[j] && (d.x & bit)) ? (int32_t)(d.y + __popc(d.x & (bit - 1u))) : -1;
        }
        if (lds_bins) {
            // 4. slot of every record inside its (tile, bin) group
            int32_t slot[kWalkItems];
            if (one_bin) {
                // one bin (at most kBinWidth survivors): a lane's slot is the
                // number of the wave's records before it (items in order,
                // lanes in order) plus the records of the waves before
                int32_t run = 0;
#pragma unroll
                for (int j = 0; j < kWalkItems; ++j) {
                    const unsigned long long m = __ballot(rk[j] >= 0);
                    slot[j] = run + lanes_below(m);
                    run += (int32_t)__popcll(m);
                }
                if (lane_id() == 0) wtot[wave_id()] = run;
                __syncthreads();
                int32_t before = 0, all = 0;
#pragma unroll
                for (int v = 0; v < kWaves; ++v) {
                    before += v < wave_id() ? wtot[v] : 0;
                    all += wtot[v];
                }
                if (tid == 0) tcount[0] = all;
#pragma unroll
                for (int j = 0; j < kWalkItems; ++j) slot[j] += before;
            } else {
                // several bins: one LDS atomic per record; the returns are
                // independent, so they pipeline (measured faster than one
                // ballot per bin and item from two bins up)
#pragma unroll
                for (int j = 0; j < kWalkItems; ++j)
                    slot[j] = rk[j] >= 0 ? atomicAdd(&tcount[rk[j] >> kBinShift], 1) : 0;
            }
            __syncthreads();
            {
                // 5. the tile's records go to its own region, grouped by bin:
                //    exclusive prefix of the bin counts, also kept in the table
                const int q = (nb + kBlock - 1) / kBlock;
                const int b0 = min(nb, q * tid), b1 = min(nb, b0 + q);
                int32_t s = 0;
                for (int b = b0; b < b1; ++b) s += tcount[b];
                int32_t all;
                int32_t at = block_excl_sum(s, red, &all);
                uint16_t* __restrict__ to = w.toff + (int64_t)t * (nb + 1);
                for (int b = b0; b < b1; ++b) {
                    const int32_t k = tcount[b];
                    tcount[b] = at;
                    to[b] = (uint16_t)at;
                    at += k;
                }
                if (tid == 0) to[nb] = (uint16_t)all;
            }
            __syncthreads();
            // 6. records
            uint16_t* __restrict__ tr = recs + (int64_t)t * kWalkTile;
#pragma unroll
            for (int j = 0; j < kWalkItems; ++j) {
                if (rk[j] >= 0) {
                    tr[tcount[rk[j] >> kBinShift] + slot[j]] = (uint16_t)(rk[j] & (kBinWidth - 1));
                    ++cross;
                }
            }
        } else {
            // bin b's region is [bin_start[b], bin_start[b + 1]): the degrees
            // of its survivors, which bound its records for a symmetric CSR.
            // Records past the end (a survivor named by more rows than its
            // degree: no valid input) are dropped and the pass is reported
            // as an invariant violation.  Every bound is at most 2m < 2^31
            // and a cursor moves by at most 2m per pass, so the unsigned
            // comparison also rejects a cursor that wrapped past INT32_MAX.
            const int32_t* __restrict__ bstart = w.bin_start;
#pragma unroll
            for (int j = 0; j < kWalkItems; ++j) {
                if (rk[j] >= 0) {
                    const int32_t b = rk[j] >> kBinShift;
                    const int32_t at = atomicAdd(&bin_cur[b], 1);
                    if ((uint32_t)at < (uint32_t)bstart[b + 1]) {
                        recs[at] = (uint16_t)(rk[j] & (kBinWidth - 1));
                    } else {
                        st->status = kStInvariant;
                    }
                    ++cross;
                }
            }
        }
        __syncthreads();
    }
    // one slot per workgroup, summed by k_walk_finish (same-address device
    // atomics from every workgroup serialise at about 15 ns each)
    const unsigned long long bc = block_sum((unsigned long long)cross, redc);
    if (tid == 0) w.wpart[blockIdx.x] = bc;
}

// ------------------------------------------------------ walk: id buckets
// Walk mode 2.  A workgroup takes groups of kIdGroupTiles consecutive walk
// tiles.  Every walked entry with a valid neighbour id becomes one record,
// the id's position inside its bucket; whether the neighbour survives is
// left to k_apply, so no entry gathers from the rank directory.  While the
// group's tiles are walked, the entries are counted per bucket in LDS; the
// counts' prefix then seeds one cursor per bucket, each entry takes its slot
// from its bucket's cursor (the records sorted by bucket in LDS), and the
// group stores them as one contiguous run (16-byte stores) with every
// bucket's (start | end << 16) in the group's column of the offset table.

__global__ __launch_bounds__(kBlock) void k_walk_ids(Work w, const int32_t* __restrict__ ci,
                                                     uint32_t n, uint32_t nnz) {
    DevState* st = w.st;
    if (st->done || st->walk_mode != 2) return;
    const int32_t nA = (int32_t)st->nA;
    const uint32_t total = (uint32_t)st->edges;
    const int32_t ntiles = st->n_tiles_walk;
    const int32_t ngroups = st->id_groups;
    const int32_t nb = st->id_nb;
    const int tid = threadIdx.x;
    constexpr uint32_t kNone = 0xFFFFFFFFu;

    // the tiles' owner tables and the group's sorted records are never live
    // at once and share their LDS
    constexpr int kOwnBytes = 2 * kWalkTile, kBasBytes = 4 * (kWalkTile + 1);
    constexpr int kPool = std::max(kOwnBytes + kBasBytes, 2 * kIdGroup);
    __shared__ __align__(16) unsigned char pool[kPool];
    uint16_t* own = reinterpret_cast<uint16_t*>(pool);
    int32_t* bas = reinterpret_cast<int32_t*>(pool + kOwnBytes);
    uint16_t* stage = reinterpret_cast<uint16_t*>(pool);
    __shared__ int32_t hist[kIdMaxBuckets];  // bucket counts, then cursors
    __shared__ int32_t red[kWaves];
    __shared__ int32_t s_row[kIdGroupTiles + 1];  // row owning each tile's first entry

    for (int32_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        for (int b = tid; b < nb; b += kBlock) hist[b] = 0;
        // the rows of the group's tiles, all loaded at once (nA - 1 past the
        // last tile of the pass)
        if (tid <= kIdGroupTiles) {
            const int32_t t = g * kIdGroupTiles + tid;
            s_row[tid] = t < ntiles ? w.tile_first[t] : nA - 1;
        }
        __syncthreads();
        uint32_t key[kIdGroupTiles][kWalkItems];  // neighbour id, or kNone
#pragma unroll
        for (int s = 0; s < kIdGroupTiles; ++s) {
#pragma unroll
            for (int j = 0; j < kWalkItems; ++j) key[s][j] = kNone;
            // every condition below is the same in the whole workgroup
            const int32_t t = g * kIdGroupTiles + s;
            if (t >= ntiles) continue;
            const uint32_t e0 = (uint32_t)t * kWalkTile;
            const int32_t len = (int32_t)min((uint32_t)kWalkTile, total - e0);
            const int32_t i0 = s_row[s];
            const int32_t ihi = s_row[s + 1];
            if (i0 < 0 || ihi >= nA || ihi < i0 || ihi - i0 + 1 > kWalkTile + 1) {
                // cannot happen for a consistent walk list; never index with it
                if (tid == 0) st->status = kStInvariant;
                continue;
            }
            const int32_t c = ihi - i0 + 1;
            int32_t rb[kWalkItems];
            tile_row_bases(w, i0, c, e0, len, rb, own, bas, red, false, [] {});
            // neighbour ids, all loads issued before any is used (clamped
            // indices; lanes past the tile end re-read its last entry)
            uint32_t u[kWalkItems];
#pragma unroll
            for (int j = 0; j < kWalkItems; ++j) {
                const uint32_t p = (uint32_t)min(j * kBlock + tid, len - 1);
                const uint32_t pos = min((uint32_t)rb[j] + e0 + p, nnz - 1u);
                u[j] = (uint32_t)__builtin_nontemporal_load(ci + pos);
            }
#pragma unroll
            for (int j = 0; j < kWalkItems; ++j) {
                if (j * kBlock + tid >= len || u[j] >= n) u[j] = kNone;  // ids outside 0..n-1
                if (u[j] != kNone) atomicAdd(&hist[u[j] >> kIdShift], 1);
                key[s][j] = u[j];
            }
            __syncthreads();  // own[] and bas[] are rebuilt for the next tile
        }
        // bucket offsets: exclusive prefix of the counts, the group's column
        // of the offset table, and the start of every bucket's cursor
        int32_t all;
        {
            const int q = (nb + kBlock - 1) / kBlock;
            const int b0 = min(nb, q * tid), b1 = min(nb, b0 + q);
            int32_t sum = 0;
            for (int b = b0; b < b1; ++b) sum += hist[b];
            int32_t at = block_excl_sum(sum, red, &all);
            // bucket-major (b * groups + g): k_apply reads a bucket's bounds
            // over consecutive groups as one coalesced run
            uint32_t* __restrict__ to = reinterpret_cast<uint32_t*>(w.toff) + g;
            for (int b = b0; b < b1; ++b) {
                const int32_t k = hist[b];
                hist[b] = at;
                to[(int64_t)b * ngroups] = (uint32_t)at | ((uint32_t)(at + k) << 16);
                at += k;
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kIdGroupTiles; ++s)
#pragma unroll
            for (int j = 0; j < kWalkItems; ++j)
                if (key[s][j] != kNone)
                    stage[atomicAdd(&hist[key[s][j] >> kIdShift], 1)] =
                        (uint16_t)(key[s][j] & (kIdWidth - 1));
        __syncthreads();
        {
            const uint4* src = reinterpret_cast<const uint4*>(stage);
            uint4* __restrict__ dst = reinterpret_cast<uint4*>(w.recs + (int64_t)g * kIdGroup);
            for (int i = tid; i < (all + 7) / 8; i += kBlock) dst[i] = src[i];
        }
        __syncthreads();  // hist[] and the pool are reused by the next group
    }
}

// Walk mode 2: the apply work items, planned after the walk.  Bucket b gets
// one item and its share of up to kTargetItems more, in proportion to the
// adjacency entries of its ids (which bound its records and track them);
// each item covers a contiguous range of the pass's record groups.
__device__ void plan_id_items(const Work& w, const int32_t* __restrict__ rp, int64_t n,
                              int32_t* red) {
    DevState* st = w.st;
    const int32_t nb = st->id_nb;
    const int64_t G = st->id_groups;
    const int64_t tot = rp[n];
    const int64_t cap = st->max_items;
    const int64_t extra = std::max<int64_t>(0, std::min<int64_t>(kTargetItems, cap - nb));
    const int q = (nb + kBlock - 1) / kBlock;
    const int b0 = std::min(nb, q * (int)threadIdx.x), b1 = std::min(nb, b0 + q);
    int32_t cnt = 0;
    for (int b = b0; b < b1; ++b) {
        const int64_t lo = (int64_t)b << kIdShift;
        const int64_t deg = rp[std::min<int64_t>(n, lo + kIdWidth)] - rp[lo];
        cnt += (int32_t)std::min<int64_t>(G, 1 + (tot > 0 ? extra * deg / tot : 0));
    }
    int32_t total;
    int32_t first = block_excl_sum(cnt, red, &total);
    if (total > cap) {  // cannot happen: nb + extra <= cap
        if (threadIdx.x == 0) {
            st->status = kStInvariant;
            st->done = 1;
            st->n_items = 0;
        }
        return;
    }
    for (int b = b0; b < b1; ++b) {
        const int64_t lo = (int64_t)b << kIdShift;
        const int64_t deg = rp[std::min<int64_t>(n, lo + kIdWidth)] - rp[lo];
        const int32_t k = (int32_t)std::min<int64_t>(G, 1 + (tot > 0 ? extra * deg / tot : 0));
        const int32_t npos = (int32_t)std::min<int64_t>(kIdWidth, n - lo);
        w.bin_items[b] = make_int2(first, k);
        for (int32_t j = 0; j < k; ++j)
            w.items[first + j] = make_int4(b, (int)(G * j / k), (int)(G * (j + 1) / k), npos);
        first += k;
    }
    if (threadIdx.x == 0) {
        st->n_items = total;
        st->apply_direct = 0;
        st->apply_next = 0;
    }
}

// Phase 0 (after the walk): sums the walk workgroups' record counts and
// completes the pass: |V|, |E|, the best graph, the next threshold and the
// apply work items; in walk mode 2 it only plans the work items.  Phase 1
// (after the degree update): in walk mode 2, sums the apply workgroups'
// counts of records that reached a survivor and completes the pass.
__global__ __launch_bounds__(kBlock) void k_walk_finish(Work w, const int32_t* __restrict__ rp,
                                                        int64_t n, int32_t parts, int32_t phase) {
    DevState* st = w.st;
    if (st->done) return;
    __shared__ int32_t red[kWaves];
    __shared__ unsigned long long redc[kWaves];
    __shared__ int32_t s_keep;
    const bool ids = st->walk_mode == 2;
    if (phase == 0 && ids) {
        plan_id_items(w, rp, n, red);
        return;
    }
    if (phase == 1 && !ids) return;
    unsigned long long c = 0;
    for (int32_t i = threadIdx.x; i < parts; i += kBlock) c += w.wpart[i];
    c = block_sum(c, redc);
    if (threadIdx.x == 0) st->cross = c;
    __syncthreads();
    finish_pass(w, &s_keep, red);
}

// ----------------------------------------------------------------- apply
// One work item = the records of one bin over a range of walk tiles (or one
// range of a bin region): count them per rank in LDS and store the counts as
// a partial row.

// Walk mode 2: an item counts its bucket's records over its range of record
// groups, then resolves every position from the bucket's rank-directory
// words (staged once): a position whose live bit is set is a survivor, and
// its count goes to the item's partial row at the position (k_reduce sums a
// bucket's rows into its survivors' degrees).  Counts that reach a survivor
// are this workgroup's part of the pass's decrements.
//
// The eight records of chunk k (records 8k .. 8k + 7 of the group) that lie
// in the run [s, e) are counted; the others go to this lane's spare counter
// past the bucket's (no branch, and no two lanes share a spare).
__device__ inline void count_chunk(uint4 q, int32_t k, int32_t s, int32_t e, int32_t* cnt) {
    const uint32_t v[4] = {q.x, q.y, q.z, q.w};
    const uint32_t spare = kIdWidth + (uint32_t)lane_id();
    const uint32_t off = (uint32_t)(k * 8 - s), len = (uint32_t)(e - s);
#pragma unroll
    for (int h = 0; h < 8; ++h) {
        const uint32_t r = (v[h >> 1] >> ((h & 1) * 16)) & (kIdWidth - 1);
        atomicAdd(&cnt[off + h < len ? r : spare], 1);
    }
}

__device__ void apply_ids(const Work& w, int32_t* cnt, uint32_t* se, uint2* sdir,
                          uint32_t* red32, unsigned long long* redc) {
    constexpr int kNW = kApplyBlock / 64;
    const DevState* st = w.st;
    const int32_t n_items = st->n_items;
    const int32_t stride = st->part_stride;
    const int64_t G = st->id_groups;
    const uint32_t* __restrict__ toff2 = reinterpret_cast<const uint32_t*>(w.toff);
    const int64_t nwords = st->id_words;
    const uint16_t* __restrict__ recs = w.recs;
    const int tid = threadIdx.x;
    unsigned long long cross = 0;
    // Items differ in size (R-MAT's hub buckets are heavy), so after its
    // first item a workgroup takes the next free one from a device counter;
    // the take is issued when an item starts and read when it ends.
    __shared__ int32_t s_next;
    for (int32_t it = blockIdx.x; it < n_items;) {
        int32_t next = 0;
        if (tid == 0)
            next = (int32_t)gridDim.x + (int32_t)atomicAdd(&w.st->apply_next, 1u);
        const int4 item = w.items[it];
        const int32_t b = item.x, npos = item.w;
        const int64_t w0 = (int64_t)b * kIdWords;
        const int32_t nw = (int32_t)std::min<int64_t>(kIdWords, nwords - w0);
        for (int i = tid; i < npos; i += kApplyBlock) cnt[i] = 0;
        for (int i = tid; i < nw; i += kApplyBlock) sdir[i] = w.dir[w0 + i];
        __syncthreads();
        for (int64_t c0 = item.y; c0 < item.z; c0 += kApplyTiles) {
            const int32_t cn = (int32_t)std::min<int64_t>(kApplyTiles, item.z - c0);
            uint32_t len = 0;
            {
                // the run bounds of up to kApplyTiles groups, every load
                // issued before any is stored (indices clamped to the last)
                constexpr int kR = kApplyTiles / kApplyBlock;
                uint32_t x[kR];
#pragma unroll
                for (int a = 0; a < kR; ++a)
                    x[a] = toff2[b * G + c0 + std::min(tid + a * kApplyBlock, cn - 1)];
#pragma unroll
                for (int a = 0; a < kR; ++a) {
                    const int32_t i = tid + a * kApplyBlock;
                    if (i < cn) {
                        se[i] = x[a];
                        len += (x[a] >> 16) - (x[a] & 0xFFFFu);
                    }
                }
            }
            // lanes per run: enough 8-record chunks, one per lane, for a
            // mean run at any alignment; the lanes of a run load adjacent
            // 16-byte chunks in one instruction.  Each group of lanes has
            // kRuns runs in flight; the rest of a longer run follows in a loop.
            const uint32_t all = block_sum<uint32_t, kNW>(len, red32);
            int lanes = 1;
            while (lanes < 64 && 8u * (uint32_t)lanes * (uint32_t)cn < all + 8u * (uint32_t)cn)
                lanes *= 2;
            const int groups = kApplyBlock / lanes, grp = tid / lanes, sub = tid % lanes;
            constexpr int kRuns = 8;
            for (int32_t i0 = grp; i0 < cn; i0 += kRuns * groups) {
                uint32_t xs[kRuns];
                uint4 q[kRuns];
#pragma unroll
                for (int a = 0; a < kRuns; ++a) {
                    // past the last run, or past a run's end, the load
                    // re-reads a chunk of the region (the run's first one)
                    // and nothing outside a run is counted; an empty run may
                    // start at the region's end
                    const int32_t i = i0 + a * groups;
                    xs[a] = i < cn ? se[i] : 0u;
                    const int32_t rs = (int32_t)(xs[a] & 0xFFFFu), re = (int32_t)(xs[a] >> 16);
                    const uint4* __restrict__ r = reinterpret_cast<const uint4*>(
                        recs + (c0 + std::min(i, cn - 1)) * (int64_t)kIdGroup);
                    const int32_t k0 = std::min(rs >> 3, kIdGroup / 8 - 1);
                    q[a] = r[(k0 + sub) * 8 < re ? k0 + sub : k0];
                }
#pragma unroll
                for (int a = 0; a < kRuns; ++a) {
                    const int32_t rs = (int32_t)(xs[a] & 0xFFFFu), re = (int32_t)(xs[a] >> 16);
                    const int32_t k = std::min(rs >> 3, kIdGroup / 8 - 1) + sub;
                    count_chunk(q[a], k, rs, re, cnt);
                    if ((k + lanes) * 8 < re) {
                        const uint4* __restrict__ r = reinterpret_cast<const uint4*>(
                            recs + (c0 + i0 + a * groups) * (int64_t)kIdGroup);
                        for (int32_t kx = k + lanes; kx * 8 < re; kx += lanes)
                            count_chunk(r[kx], kx, rs, re, cnt);
                    }
                }
            }
            __syncthreads();  // se is reloaded for the next groups; counts are done
        }
        // every live position's count goes to the item's partial row (stores
        // only: no round trip holds up the item); k_reduce applies the rows
        for (int p = tid; p < npos; p += kApplyBlock) {
            const uint2 d = sdir[p >> 5];
            if (d.x & (1u << (p & 31))) {
                const int32_t c = cnt[p];
                cross += (uint32_t)c;
                w.partial[(int64_t)it * stride + p] = c;
            }
        }
        if (tid == 0) s_next = next;
        __syncthreads();  // cnt and sdir are reused by the next item; s_next is set
        it = s_next;
    }
    const unsigned long long all = block_sum<unsigned long long, kNW>(cross, redc);
    if (tid == 0) w.wpart[blockIdx.x] = all;
}

__global__ __launch_bounds__(kApplyBlock) void k_apply(Work w) {
    const DevState* st = w.st;
    __shared__ int32_t cnt[kBinWidth + 64];  // (walk mode 2: one spare counter per lane)
    __shared__ uint32_t se[kApplyTiles];  // (start | end << 16) of a tile's run
    __shared__ uint2 sdir[kIdWords];
    __shared__ uint32_t red32[kApplyBlock / 64];
    __shared__ unsigned long long redc[kApplyBlock / 64];
    const int32_t mode = st->walk_mode;
    if (mode == 2) {
        apply_ids(w, cnt, se, sdir, red32, redc);
        return;
    }
    const int32_t n_items = st->n_items;
    if (n_items == 0) return;
    const int32_t stride = st->part_stride;
    const int64_t tstride = st->toff_stride;
    const uint16_t* __restrict__ recs = w.recs;
    // few records: the item subtracts its nonzero counts from the degrees
    // itself (one device atomic per rank and item), so that no partial row
    // is written and k_reduce has nothing to do
    const bool direct = st->apply_direct != 0;
    int32_t* __restrict__ deg = deg_in(w, st->pass);  // the pass counter has advanced
    const int lanes = st->apply_lanes;
    const int groups = kApplyBlock / lanes;
    const int grp = threadIdx.x / lanes;
    const int sub = threadIdx.x % lanes;
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 item = w.items[it];
        const int32_t ranks = item.w;
        for (int i = threadIdx.x; i < ranks; i += kApplyBlock) cnt[i] = 0;
        __syncthreads();
        if (mode == 0) {
            // groups of `lanes` threads walk one tile's run of this bin's
            // records; the runs' bounds of up to kApplyTiles tiles are
            // loaded into LDS first, all at once, so that no group waits
            // on a bounds load between two runs
            for (int64_t c0 = item.y; c0 < item.z; c0 += kApplyTiles) {
                const int32_t cn = (int32_t)std::min<int64_t>(kApplyTiles, item.z - c0);
                for (int32_t i = threadIdx.x; i < cn; i += kApplyBlock) {
                    const uint16_t* __restrict__ o = w.toff + (c0 + i) * tstride + item.x;
                    se[i] = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
                }
                __syncthreads();
                for (int32_t i = grp; i < cn; i += groups) {
                    const int32_t s = (int32_t)(se[i] & 0xFFFFu), e = (int32_t)(se[i] >> 16);
                    const uint16_t* __restrict__ r = recs + (c0 + i) * (int64_t)kWalkTile;
                    for (int32_t x0 = s + sub; x0 < e; x0 += kApplyBatch * lanes) {
                        // issue the batch's loads before any count
                        uint32_t v[kApplyBatch];
#pragma unroll
                        for (int k = 0; k < kApplyBatch; ++k) {
                            const int32_t x = x0 + k * lanes;
                            v[k] = x < e ? (uint32_t)r[x] : 0xFFFFFFFFu;
                        }
#pragma unroll
                        for (int k = 0; k < kApplyBatch; ++k)
                            if (v[k] != 0xFFFFFFFFu) atomicAdd(&cnt[v[k]], 1);
                    }
                }
                __syncthreads();  // se is reloaded for the next tiles
            }
        } else {
            int64_t e = (int64_t)item.y + threadIdx.x;
            const int64_t z = item.z;
            for (; e + 3 * kApplyBlock < z; e += 4 * kApplyBlock) {
                const uint32_t r0 = recs[e], r1 = recs[e + kApplyBlock];
                const uint32_t r2 = recs[e + 2 * kApplyBlock], r3 = recs[e + 3 * kApplyBlock];
                atomicAdd(&cnt[r0], 1);
                atomicAdd(&cnt[r1], 1);
                atomicAdd(&cnt[r2], 1);
                atomicAdd(&cnt[r3], 1);
            }
            for (; e < z; e += kApplyBlock) atomicAdd(&cnt[recs[e]], 1);
        }
        __syncthreads();
        if (direct) {
            const int64_t rank0 = (int64_t)item.x << kBinShift;
            for (int i = threadIdx.x; i < ranks; i += kApplyBlock) {
                const int32_t c = cnt[i];
                if (c)
                    __hip_atomic_fetch_sub(deg + rank0 + i, c, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            int32_t* __restrict__ out = w.partial + (int64_t)it * stride;
            for (int i = threadIdx.x; i < ranks; i += kApplyBlock) out[i] = cnt[i];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- reduce
// degree[r] -= sum of the partial rows of r's bin, for every survivor rank r
// of the pass just finished.  64 consecutive ranks share a bin.

__global__ __launch_bounds__(kBlock) void k_reduce(Work w) {
    const DevState* st = w.st;
    if (st->n_items == 0 || st->apply_direct) return;
    const int64_t nL = st->nL;
    const int32_t stride = st->part_stride;
    if (st->walk_mode == 2) {
        // walk mode 2: every survivor gets the sum of its bucket's items'
        // partial rows at its position; the pass has not advanced yet
        int32_t* __restrict__ deg = deg_out(w, st->pass);
        const int32_t* __restrict__ lst = live_out(w, st->pass);
        for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < nL;
             r += (int64_t)gridDim.x * kBlock) {
            const int32_t v = lst[r];
            const int2 bi = w.bin_items[v >> kIdShift];
            const int32_t* __restrict__ p =
                w.partial + (int64_t)bi.x * stride + (v & (kIdWidth - 1));
            int32_t sum = 0;
            for (int32_t j = 0; j < bi.y; ++j) sum += p[(int64_t)j * stride];
            if (sum) deg[r] -= sum;
        }
        return;
    }
    // `lanes` lanes of a wave share one rank (1..16); within the wave the
    // 64 / lanes ranks are consecutive, so each partial row is read in runs
    const int lanes = st->reduce_lanes;
    int32_t* __restrict__ deg = deg_in(w, st->pass);  // the pass counter has advanced
    const int ranks_per_wave = 64 / lanes;
    const int64_t per_block = (int64_t)kWaves * ranks_per_wave;
    const int64_t ntasks = (nL + per_block - 1) / per_block;
    const int sub = lane_id() / ranks_per_wave;
    const int rr = lane_id() % ranks_per_wave;
    for (int64_t task = blockIdx.x; task < ntasks; task += gridDim.x) {
        const int64_t r = task * per_block + (int64_t)wave_id() * ranks_per_wave + rr;
        // every load below is unconditional, at a clamped index, and only
        // counted when in range (a load under a condition is waited for at
        // once): the rank's degree with its partial rows, 8 rows per lane
        // in flight
        const int64_t rc = std::min<int64_t>(r, nL - 1);
        const int2 bi = w.bin_items[rc >> kBinShift];
        const int32_t d0 = deg[rc];
        int32_t sum = 0;
        if (r < nL && bi.y > 0) {
            const int32_t* __restrict__ p =
                w.partial + (int64_t)bi.x * stride + (r & (kBinWidth - 1));
            for (int32_t i = sub; i < bi.y; i += 8 * lanes) {
                int32_t v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    v[k] = p[(int64_t)std::min(i + k * lanes, bi.y - 1) * stride];
#pragma unroll
                for (int k = 0; k < 8; ++k) sum += i + k * lanes < bi.y ? v[k] : 0;
            }
        }
        for (int off = ranks_per_wave; off < 64; off <<= 1) sum += __shfl_xor(sum, off, 64);
        if (sub == 0 && r < nL && sum) deg[r] = d0 - sum;
    }
}

// --------------------------------------------------------------- extract
// S~ = { v : removed_at[v] > best_pass }, ascending.

// S~ = { v : removed_at[v] > best_pass }, or with `flag` (CBDS-P) also
// every v with flag[v] != 0.
__global__ __launch_bounds__(kBlock) void k_extract_count(Work w, int64_t n,
                                                          const int32_t* __restrict__ flag) {
    const DevState* st = w.st;
    if (!st->done || st->status != kStOk) return;
    const int32_t bp = st->best_pass;
    const int64_t ntiles = (n + kMarkTile - 1) / kMarkTile;
    __shared__ uint32_t red[kWaves];
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t base = t * kMarkTile + (int64_t)threadIdx.x * kMarkItems;
        int32_t ra[kMarkItems], fl[kMarkItems];
        load8(w.removed_at, base, n, 0, ra);
        if (flag) {
            load8(flag, base, n, 0, fl);
        } else {
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) fl[j] = 0;
        }
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < kMarkItems; ++j)
            if (base + j < n && (ra[j] > bp || fl[j])) ++c;
        const uint32_t tc = block_sum(c, red);
        if (threadIdx.x == 0) w.tiles[2 * t] = make_int4((int)tc, 0, 0, 0);
    }
}

__global__ __launch_bounds__(kBlock) void k_extract_scatter(Work w, int64_t n,
                                                            int32_t* __restrict__ best,
                                                            const int32_t* __restrict__ flag) {
    const DevState* st = w.st;
    if (!st->done || st->status != kStOk) return;
    const int32_t bp = st->best_pass;
    const int64_t ntiles = (n + kMarkTile - 1) / kMarkTile;
    __shared__ uint32_t red[kWaves];
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t base = t * kMarkTile + (int64_t)threadIdx.x * kMarkItems;
        int32_t ra[kMarkItems], fl[kMarkItems];
        load8(w.removed_at, base, n, 0, ra);
        if (flag) {
            load8(flag, base, n, 0, fl);
        } else {
#pragma unroll
            for (int j = 0; j < kMarkItems; ++j) fl[j] = 0;
        }
        uint32_t keep = 0, c = 0;
#pragma unroll
        for (int j = 0; j < kMarkItems; ++j)
            if (base + j < n && (ra[j] > bp || fl[j])) {
                keep |= 1u << j;
                ++c;
            }
        uint32_t tot;
        const uint32_t ex = block_excl_sum(c, red, &tot);
        int64_t pos = (int64_t)w.tiles[2 * t].x + ex;
#pragma unroll
        for (int j = 0; j < kMarkItems; ++j)
            if ((keep >> j & 1u) && pos < n) best[pos++] = (int32_t)(base + j);
    }
}

// S~ when the best graph is the whole graph (best pass 0): 0..n-1.  Any
// other S~ is a pass's survivor list, which k_mark_count has copied.
__global__ __launch_bounds__(kBlock) void k_extract_iota(Work w, int64_t n,
                                                         int32_t* __restrict__ best) {
    DevState* st = w.st;
    if (!st->done || st->status != kStOk || st->best_pass != 0) return;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride)
        best[v] = (int32_t)v;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->best_count = n;
}

// ================================================================ CBDS-P
// Phase 2 of Algorithm 2 (Section 3.2), after the k-core levels.  removed_at
// holds every vertex's core number; the densest core is C_K = { v : core(v)
// > cut } with cut = K - 1 = best_pass, |E(C_K)| = best_E, |C_K| = best_S,
// and rho = best_E / best_S.  All tests are exact cross-multiplications.

// Outside vertices with core(v) > rho (the only ones that can have more
// than rho neighbours in C_K, since a vertex's neighbours inside a core it
// is not part of number at most its core number) go to `elist`.  Also
// clears the legitimate flags.
__global__ __launch_bounds__(kBlock) void k_cbds_eligible(Work w, int64_t n, int32_t* flag,
                                                          int32_t* elist) {
    DevState* st = w.st;
    if (!st->done || st->status != kStOk) return;
    const int32_t cut = st->best_pass;
    const int64_t me = st->best_E, mv = st->best_S;
    for (int64_t b = (int64_t)blockIdx.x * kBlock; b < n; b += (int64_t)gridDim.x * kBlock) {
        const int64_t v = b + threadIdx.x;
        bool elig = false;
        if (v < n) {
            flag[v] = 0;
            const int32_t c = w.removed_at[v];
            elig = c <= cut && (int64_t)c * mv > me;
        }
        // one atomic per wave
        const unsigned long long mask = __ballot(elig);
        if (mask) {
            uint32_t at = 0;
            if (lane_id() == 0) at = atomicAdd(&st->cb_nelig, (uint32_t)__popcll(mask));
            at = __shfl(at, 0, 64);
            if (elig) elist[at + lanes_below(mask)] = (int32_t)v;
        }
    }
}

// legits(v) = neighbours of v inside C_K, one wave per eligible vertex;
// v is legitimate when legits(v) > rho.
__global__ __launch_bounds__(kBlock) void k_cbds_legits(Work w, const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci, int64_t n,
                                                        int32_t* flag, const int32_t* elist,
                                                        int32_t* llist) {
    DevState* st = w.st;
    if (!st->done || st->status != kStOk) return;
    const int32_t cut = st->best_pass;
    const int64_t me = st->best_E, mv = st->best_S;
    const int64_t ne = st->cb_nelig;
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    for (int64_t i = (int64_t)blockIdx.x * kWaves + wave_id(); i < ne; i += waves) {
        const int32_t v = elist[i];
        const int32_t r0 = rp[v], r1 = rp[v + 1];
        uint32_t cnt = 0;
        for (int32_t e = r0 + lane_id(); e < r1; e += 64) {
            const int32_t u = ci[e];
            cnt += (uint64_t)(int64_t)u < (uint64_t)n && w.removed_at[u] > cut;
        }
        cnt = wave_sum(cnt);
        if (lane_id() == 0 && (int64_t)cnt * mv > me) {
            flag[v] = 1;
            atomicAdd(&st->cb_sumlegit, (unsigned long long)cnt);
            llist[atomicAdd(&st->cb_nlegit, 1u)] = v;
        }
    }
}

// Edges among legitimate vertices, each counted at its smaller end.
__global__ __launch_bounds__(kBlock) void k_cbds_pairs(Work w, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, int64_t n,
                                                       const int32_t* flag, const int32_t* llist) {
    DevState* st = w.st;
    if (!st->done || st->status != kStOk) return;
    const int64_t nl = st->cb_nlegit;
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    for (int64_t i = (int64_t)blockIdx.x * kWaves + wave_id(); i < nl; i += waves) {
        const int32_t v = llist[i];
        const int32_t r0 = rp[v], r1 = rp[v + 1];
        uint32_t cnt = 0;
        for (int32_t e = r0 + lane_id(); e < r1; e += 64) {
            const int32_t u = ci[e];
            cnt += u > v && (uint64_t)(int64_t)u < (uint64_t)n && flag[u] != 0;
        }
        cnt = wave_sum(cnt);
        if (lane_id() == 0 && cnt) atomicAdd(&st->cb_el, (unsigned long long)cnt);
    }
}

// ============================================================ device tail
// The passes of a peel that the host did not enqueue as kernels: one
// workgroup runs Algorithm 1's loop (Section 3.1) on the device until the
// graph is empty, the pass watchdog trips or an invariant fails.  Each pass
// is the same step sequence as the seven-kernel pass, with workgroup
// barriers in place of kernel boundaries:
//
//   copy     when the previous pass set the best graph, its survivor list
//            (this pass's live list, ascending) becomes S~;
//   mark     every live vertex with degree <= T_k fails (removal pass,
//            live bit cleared); a stable compaction writes the survivors
//            (id, degree) and the walk list (row start, prefix of row
//            lengths) of the failures with degree > 0;
//   ranks    the rank directory of the survivors (first rank per 32-vertex
//            word);
//   walk     the walk list's entries in tiles of kTailTile: every entry
//            whose neighbour survives decrements that survivor's degree
//            (one device atomic);
//   finish   |V|, |E| = |E| - cross - intra / 2, the best graph (strict),
//            the next threshold, the watchdog, the trace record.
//
// Data that another thread of the workgroup wrote in this kernel (lists,
// degrees, the rank directory, the walk list) is read with L1-bypassing
// loads, and degrees and live bits are changed with device atomics.

constexpr int kTailBlock = 1024;
constexpr int kTailWaves = kTailBlock / 64;
constexpr int kTailItems = 8;                       // walk entries per thread and tile
constexpr int kTailTile = kTailBlock * kTailItems;  // walk entries per tile

__device__ inline int32_t ld_co(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint2 ld_co(const uint2* p) {
    const unsigned long long x = __hip_atomic_load(
        reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
        __HIP_MEMORY_SCOPE_AGENT);
    return make_uint2((uint32_t)x, (uint32_t)(x >> 32));
}

// Last index i in [lo, hi) with aoff[i] <= target, given aoff[lo] <= target
// and aoff strictly increasing (every walked row has an entry).  Run by one
// whole wave: each round probes 64 evenly spaced rows at once.
__device__ inline int32_t wave_find_row(const int32_t* aoff, int32_t lo32, int32_t hi32,
                                        int32_t target) {
    const int lane = lane_id();
    int64_t lo = lo32, hi = hi32;
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t probe = lo + (int64_t)lane * step;
        const bool ok = probe < hi && ld_co(aoff + probe) <= target;
        const int k = (int)__popcll(__ballot(ok)) - 1;  // ok lanes are a prefix; lane 0 is ok
        lo = lo + (int64_t)max(k, 0) * step;
        hi = min(hi, lo + step);
    }
    return (int32_t)lo;
}

__global__ __launch_bounds__(kTailBlock) void k_tail(Work w, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, int64_t n,
                                                     int64_t nnz, int32_t* __restrict__ best) {
    DevState* st = w.st;
    const int tid = threadIdx.x;
    __shared__ uint32_t red32[kTailWaves];
    __shared__ unsigned long long red64[kTailWaves];
    __shared__ int32_t s_aoff[kTailTile + 1], s_arow[kTailTile + 1];
    __shared__ int32_t s_r0, s_r1;
    __shared__ int32_t s_pass, s_T, s_done, s_best_pass;
    __shared__ int64_t s_S;
    if (tid == 0) {
        s_done = st->done;
        s_pass = st->pass;
        s_T = st->T;
        s_S = st->S;
        s_best_pass = st->best_pass;
    }
    __syncthreads();
    while (!s_done) {
        const int32_t pass = s_pass;
        const int32_t T = s_T;
        const int64_t S = s_S;
        const int32_t* L = live_in(w, pass);  // pass >= 2: pass 1 always runs as kernels
        int32_t* D = deg_in(w, pass);
        int32_t* Lo = live_out(w, pass);
        int32_t* Do = deg_out(w, pass);

        // copy: S~ is the survivor list of the previous pass
        if (best && s_best_pass == pass - 1) {
            for (int64_t i = tid; i < S; i += kTailBlock) best[i] = ld_co(L + i);
            if (tid == 0) st->best_count = S;
        }

        // mark and stable compaction, one live-list entry per thread and round
        int64_t offL = 0, offA = 0, offE = 0;
        unsigned long long sumF = 0;  // degrees of the failures
        for (int64_t c0 = 0; c0 < S; c0 += kTailBlock) {
            const int64_t i = c0 + tid;
            int32_t v = -1, d = 0, len = 0;
            if (i < S) {
                v = ld_co(L + i);
                d = ld_co(D + i);
                if ((uint64_t)(int64_t)v >= (uint64_t)n) v = -1;
            }
            const bool fail = v >= 0 && d <= T;
            const bool walk = fail && d > 0;
            if (walk) len = rp[v + 1] - rp[v];
            if (fail) {
                w.removed_at[v] = pass;
                atomicAnd(&w.dir[v >> 5].x, ~(1u << (v & 31)));
                sumF += (unsigned long long)(int64_t)d;
            }
            uint32_t tot_la, tot_e;
            const uint32_t ex_la = block_excl_sum<uint32_t, kTailWaves>(
                (v >= 0 && !fail ? 1u : 0u) | (walk ? 1u << 16 : 0u), red32, &tot_la);
            const uint32_t ex_e = block_excl_sum<uint32_t, kTailWaves>((uint32_t)len, red32, &tot_e);
            if (v >= 0 && !fail) {
                const int64_t p = offL + (ex_la & 0xFFFFu);
                if (p < n) {
                    Lo[p] = v;
                    Do[p] = d;
                }
            } else if (walk) {
                const int64_t p = offA + (ex_la >> 16);
                if (p < n) {
                    w.arow[p] = rp[v];
                    w.aoff[p] = (int32_t)(offE + ex_e);
                }
            }
            offL += tot_la & 0xFFFFu;
            offA += tot_la >> 16;
            offE += tot_e;
        }
        const int64_t nL = offL, nA = offA, E_walk = offE;
        sumF = block_sum<unsigned long long, kTailWaves>(sumF, red64);

        // rank directory: the first survivor of every 32-vertex word
        for (int64_t r = tid; r < nL; r += kTailBlock) {
            const int32_t v = ld_co(Lo + r);
            const int32_t pv = r > 0 ? ld_co(Lo + r - 1) : -1;
            if (r == 0 || (pv >> 5) != (v >> 5)) w.dir[v >> 5].y = (uint32_t)r;
        }
        __syncthreads();

        // walk (nothing to decrement when no vertex survives)
        unsigned long long cross = 0;
        const int32_t* __restrict__ aoff = w.aoff;
        const int32_t* __restrict__ arow = w.arow;
        int32_t rlo = 0;
        for (int64_t t0 = 0; nL > 0 && t0 < E_walk; t0 += kTailTile) {
            const int32_t tlen = (int32_t)min<int64_t>(kTailTile, E_walk - t0);
            if (tid < 64) {
                const int32_t r0 = wave_find_row(aoff, rlo, (int32_t)nA, (int32_t)t0);
                const int32_t r1 = wave_find_row(aoff, r0, (int32_t)nA, (int32_t)(t0 + tlen - 1));
                if (tid == 0) {
                    s_r0 = r0;
                    s_r1 = r1;
                }
            }
            __syncthreads();
            // at most tlen rows: every walked row has an entry (its degree, at
            // most its length, is positive), so row starts strictly increase
            const int32_t r0 = s_r0, nr = min(s_r1 - s_r0 + 1, kTailTile + 1);
            for (int32_t k = tid; k < nr; k += kTailBlock) {
                s_aoff[k] = ld_co(aoff + r0 + k);
                s_arow[k] = ld_co(arow + r0 + k);
            }
            __syncthreads();
            for (int32_t k = tid; k < tlen; k += kTailBlock) {
                const int32_t e = (int32_t)t0 + k;
                int32_t lo = 0, hi = nr;  // last row with s_aoff <= e
                while (hi - lo > 1) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (s_aoff[mid] <= e) lo = mid; else hi = mid;
                }
                const int64_t pos = min<int64_t>((int64_t)s_arow[lo] + (e - s_aoff[lo]), nnz - 1);
                const int32_t u = ci[pos];
                if ((uint64_t)(int64_t)u < (uint64_t)n) {
                    const uint2 dw = ld_co(w.dir + (u >> 5));
                    const uint32_t bit = 1u << (u & 31);
                    if (dw.x & bit) {
                        const uint32_t rank = dw.y + __popc(dw.x & (bit - 1u));
                        if ((int64_t)rank < nL)
                            __hip_atomic_fetch_sub(Do + rank, 1, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                        ++cross;
                    }
                }
            }
            rlo = s_r1;
            __syncthreads();  // s_aoff / s_arow are restaged for the next tile
        }
        cross = block_sum<unsigned long long, kTailWaves>(cross, red64);

        // finish (one thread), as the seven-kernel pass does
        if (tid == 0) {
            const int64_t S_in = S, E_in = st->E, S_out = nL;
            const int64_t intra = (int64_t)sumF - (int64_t)cross;
            const int64_t E_out = E_in - (int64_t)cross - intra / 2;
            int32_t done = 0;
            if (st->status != kStOk || intra < 0 || (intra & 1) || E_out < 0 ||
                (S_out == 0 && E_out != 0)) {
                if (st->status == kStOk) st->status = kStInvariant;
                done = 1;
            } else {
                if (pass <= st->trace_cap) {
                    PassRecord r;
                    r.s_in = S_in;
                    r.e_in = E_in;
                    r.thresh = T;
                    r.removed = S_in - S_out;
                    r.cross = (int64_t)cross;
                    r.intra = intra;
                    r.walked = S_out > 0 ? E_walk : 0;
                    r.s_out = S_out;
                    r.e_out = E_out;
                    w.trace[pass - 1] = r;
                }
                st->tot_walked += S_out > 0 ? E_walk : 0;
                st->tot_cross += (int64_t)cross;
                st->tot_live += S_in;
                st->tot_alist += nA;
                if (S_out > 0 && E_out * st->best_S > st->best_E * S_out) {
                    st->best_E = E_out;
                    st->best_S = S_out;
                    st->best_pass = pass;
                }
                st->S = S_out;
                st->E = E_out;
                st->nL = S_out;
                if (S_out == 0) {
                    done = 1;
                } else if (pass + 1 > st->max_pass) {
                    st->status = kStWatchdog;
                    done = 1;
                } else {
                    st->T = pass_threshold(E_out, S_out, st->eps_num, st->eps_den);
                    st->pass = pass + 1;
                }
            }
            if (done) st->done = 1;
            s_done = done;
            s_pass = st->pass;
            s_T = st->T;
            s_S = st->S;
            s_best_pass = st->best_pass;
        }
        __syncthreads();
    }
}

// The device result of dsg_peel_async for the graph with no vertex.
__global__ void k_async_empty(dsg_batch_result* out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    dsg_batch_result r;
    r.dens_num = r.dens_den = r.best_size = 0;
    r.passes = r.best_pass = 0;
    r.status = DSG_OK;
    r.reserved = 0;
    *out = r;
}

// The device result of a peel whose passes all ran without the host
// (dsg_peel_async): the status, the density of S~ and the pass counts.
__global__ void k_async_result(Work w, dsg_batch_result* out, int32_t extracted) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const DevState* st = w.st;
    int32_t status = DSG_OK;
    if (!st->done) status = DSG_EINTERNAL;  // cannot happen: the tail runs to the end
    else if (st->status == kStBadRowPtr) status = DSG_EINVAL;
    else if (st->status != kStOk) status = DSG_EINTERNAL;
    else if (extracted && st->best_count != st->best_S) status = DSG_EINTERNAL;
    dsg_batch_result r;
    r.dens_num = status == DSG_OK ? st->best_E : 0;
    r.dens_den = status == DSG_OK ? st->best_S : 0;
    r.passes = st->pass;
    r.best_pass = st->best_pass;
    r.best_size = status == DSG_OK && extracted ? st->best_S : 0;
    r.status = status;
    r.reserved = 0;
    *out = r;
}

// ================================================================== host

namespace {

struct DevInfo {
    int cus = 0;
    int walk_blocks_per_cu = 0;
    int walk_ids_blocks_per_cu = 0;
    int apply_blocks_per_cu = 0;
    bool ready = false;
};

std::mutex g_info_mu;
DevInfo g_info[64];

hipError_t device_info(DevInfo* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_info_mu);
    DevInfo& di = g_info[dev];
    if (!di.ready) {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        int per = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_walk, kBlock, 0);
        if (e != hipSuccess) return e;
        int per_apply = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_apply, k_apply, kApplyBlock, 0);
        if (e != hipSuccess) return e;
        int per_ids = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_ids, k_walk_ids, kBlock, 0);
        if (e != hipSuccess) return e;
        di.cus = cus;
        // more than 6 resident walk workgroups per CU measured slower (the
        // rank-directory gathers of extra tiles evict each other from L2)
        di.walk_blocks_per_cu = std::max(std::min(per, 6), 1);
        di.apply_blocks_per_cu = std::max(per_apply, 1);
        di.walk_ids_blocks_per_cu = std::max(per_ids, 1);
        di.ready = true;
    }
    *out = di;
    return hipSuccess;
}

inline int64_t mark_tiles(int64_t n) { return (n + kMarkTile - 1) / kMarkTile + 1; }
inline int64_t walk_tiles(int64_t m) { return (2 * m + kWalkTile - 1) / kWalkTile + 1; }
inline int64_t max_bins(int64_t n) { return (n + kBinWidth - 1) / kBinWidth + 1; }
inline int64_t id_groups(int64_t m) { return (2 * m + kIdGroup - 1) / kIdGroup + 1; }
// neighbour-id buckets of walk mode 2, or 0 where the graph has too many ids
inline int64_t id_buckets(int64_t n) {
    const int64_t nb = (n + kIdWidth - 1) / kIdWidth;
    return nb <= kIdMaxBuckets ? nb : 0;
}
// Whether a peel's passes may take walk mode 2 (the tile scan decides per
// pass): never with forced bin regions or when the caller turns it off,
// otherwise when the flag asks for it, or when more than kFiltBits vertices
// can survive a pass and a pass can walk kIdMinEntries entries.
inline bool ids_allowed(int64_t n, int64_t m, const dsg_launch* launch) {
    const int32_t f = launch ? launch->flags : 0;
    if ((f & (DSG_LAUNCH_BIN_REGIONS | DSG_LAUNCH_NO_ID_BUCKETS)) || id_buckets(n) == 0)
        return false;
    return (f & DSG_LAUNCH_ID_BUCKETS) || (n > kFiltBits && 2 * m >= kIdMinEntries);
}
inline int64_t part_stride(int64_t n) {
    return std::min<int64_t>(kBinWidth, std::max<int64_t>(n, 1));
}
// Work items per pass.  Per-tile records: nb * min(tiles, kTargetItems / nb)
// items (at least nb), nb <= kNbLds.  Bin regions: every bin with records
// has at most one item shorter than the chunk, and the chunk is at least
// kChunkMin and at least records / kTargetItems, with records <= 2m.
inline int64_t max_items(int64_t n, int64_t m) {
    const int64_t nb = max_bins(n);
    const int64_t tile_items =
        std::min<int64_t>(std::max<int64_t>(kTargetItems, std::min<int64_t>(nb, kNbLds)),
                          nb * walk_tiles(m));
    const int64_t bin_items =
        nb + std::min<int64_t>(kTargetItems, (2 * m + kChunkMin - 1) / kChunkMin) + 1;
    return std::max(tile_items, bin_items);
}

struct Layout {
    size_t st, rem, dir, l0, l1, d0, d1, arow, aoff, tfirst, tiles, bstart, bcur, bitems, items,
        partial, recs, toff, filt, wpart, trace, total;
};

Layout layout(int64_t n, int64_t m) {
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const int64_t nb = max_bins(n);
    const int64_t ni = max_items(n, m);
    L.st = take(sizeof(DevState));
    L.rem = take(4 * (size_t)n);
    L.dir = take(8 * (size_t)((n + 31) / 32));
    L.l0 = take(4 * (size_t)n);
    L.l1 = take(4 * (size_t)n);
    L.d0 = take(4 * (size_t)n);
    L.d1 = take(4 * (size_t)n);
    L.arow = take(4 * (size_t)n);
    L.aoff = take(4 * (size_t)(n + 1));
    L.tfirst = take(4 * (size_t)walk_tiles(m));
    L.tiles = take(2 * sizeof(int4) * (size_t)mark_tiles(n));
    L.bstart = take(4 * (size_t)nb);
    L.bcur = take(4 * (size_t)nb);
    L.bitems = take(8 * (size_t)nb);
    L.items = take(sizeof(int4) * (size_t)ni);
    L.partial = take(4 * (size_t)ni * (size_t)part_stride(n));
    // per-tile regions and offsets, or per-group ones in walk mode 2
    L.recs = take(2 * (size_t)std::max<int64_t>(walk_tiles(m) * kWalkTile, id_groups(m) * kIdGroup));
    L.toff = take(std::max<size_t>(2 * (size_t)walk_tiles(m) * (std::min<int64_t>(nb, kNbLds) + 1),
                                   4 * (size_t)id_groups(m) * id_buckets(n)));
    L.filt = take(4 * (size_t)kFiltWords);
    L.wpart = take(8 * (size_t)kMaxWalkGrid);
    L.trace = take(sizeof(PassRecord) * (size_t)kTraceCap);
    L.total = o;
    return L;
}


thread_local DevState* t_host_state = nullptr;
// the tile scan's progress word (pinned, coherent host memory)
thread_local int64_t* t_progress = nullptr;

// Waits until the progress word reaches `want` and returns it; returns -1
// once the stream has no work left or has failed without that, so that the
// wait always ends.  The stream is queried only after 20 ms without the
// post: a query adds a marker to the stream, which costs every pass a gap.
static int64_t wait_progress(const int64_t* p, int64_t want, hipStream_t s) {
    auto last = std::chrono::steady_clock::now();
    for (uint32_t spin = 1;; ++spin) {
        const int64_t v = __atomic_load_n(p, __ATOMIC_ACQUIRE);
        if (v >= want) return v;
        if ((spin & 1023) == 0) {
            const auto now = std::chrono::steady_clock::now();
            if (now - last > std::chrono::milliseconds(20)) {
                last = now;
                if (hipStreamQuery(s) != hipErrorNotReady) {
                    const int64_t u = __atomic_load_n(p, __ATOMIC_ACQUIRE);
                    return u >= want ? u : -1;
                }
            }
        }
        __builtin_ia32_pause();
    }
}

enum { kKindInit = 0, kKindMark = 1, kKindWalk = 2, kKindApply = 3, kKindExtract = 4 };

struct EventLog {
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    bool on = false;
    hipStream_t s = nullptr;
    hipError_t begin(int k) {
        if (!on) return hipSuccess;
        hipEvent_t a;
        hipError_t e = hipEventCreateWithFlags(&a, hipEventDisableSystemFence);
        if (e != hipSuccess) return e;
        ev.push_back(a);
        kind.push_back(k);
        return hipEventRecord(a, s);
    }
    hipError_t end() {
        if (!on) return hipSuccess;
        hipEvent_t b;
        hipError_t e = hipEventCreateWithFlags(&b, hipEventDisableSystemFence);
        if (e != hipSuccess) return e;
        ev.push_back(b);
        return hipEventRecord(b, s);
    }
    ~EventLog() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

}  // namespace

}  // namespace dsg

using namespace dsg;

#define DSG_HIP(expr)                         \
    do {                                      \
        hipError_t _e = (expr);               \
        if (_e != hipSuccess) {               \
            rc = map_hip(_e);                 \
            goto done;                        \
        }                                     \
    } while (0)

extern "C" {

int32_t dsg_version(void) { return 2; }

const char* dsg_strerror(int32_t status) {
    switch (status) {
        case DSG_OK: return "ok";
        case DSG_EINVAL: return "invalid argument or input outside the CSR contract";
        case DSG_EOVERFLOW: return "sizes or eps outside the exact integer range";
        case DSG_ENOMEM: return "device memory allocation failed";
        case DSG_EDEVICE: return "HIP runtime error";
        case DSG_EINTERNAL: return "pass watchdog or edge-count invariant tripped";
        default: return "unknown status";
    }
}

size_t dsg_workspace_bytes(int64_t n, int64_t m) {
    if (check_sizes(n, m, 0, 1) != DSG_OK) return 0;
    return layout(n, m).total;
}

}  // extern "C"

namespace {

// Pointers of a workspace laid out by layout(n, m); removed_at is the
// caller's array when given.
Work make_work(char* base, const Layout& L, int32_t* removed_at) {
    Work w;
    w.st = (DevState*)(base + L.st);
    w.removed_at = removed_at ? removed_at : (int32_t*)(base + L.rem);
    w.dir = (uint2*)(base + L.dir);
    w.list0 = (int32_t*)(base + L.l0);
    w.list1 = (int32_t*)(base + L.l1);
    w.deg0 = (int32_t*)(base + L.d0);
    w.deg1 = (int32_t*)(base + L.d1);
    w.arow = (int32_t*)(base + L.arow);
    w.aoff = (int32_t*)(base + L.aoff);
    w.tile_first = (int32_t*)(base + L.tfirst);
    w.tiles = (int4*)(base + L.tiles);
    w.bin_start = (int32_t*)(base + L.bstart);
    w.bin_cur = (int32_t*)(base + L.bcur);
    w.bin_items = (int2*)(base + L.bitems);
    w.items = (int4*)(base + L.items);
    w.partial = (int32_t*)(base + L.partial);
    w.recs = (uint16_t*)(base + L.recs);
    w.toff = (uint16_t*)(base + L.toff);
    w.filt = (uint32_t*)(base + L.filt);
    w.wpart = (unsigned long long*)(base + L.wpart);
    w.trace = (PassRecord*)(base + L.trace);
    w.progress = nullptr;
    return w;
}

// Grid sizes of one peel's kernels.
struct Grids {
    unsigned mark, walk, init, apply, reduce, walk_ids;
    bool ids;  // the passes may take walk mode 2: its kernels are enqueued
};

Grids default_grids(const DevInfo& di, int64_t n, int64_t m, const dsg_launch* launch) {
    Grids gr;
    const int64_t mt = mark_tiles(n) - 1;
    const int64_t wt = std::max<int64_t>(walk_tiles(m) - 1, 1);
    const int64_t mg = launch && launch->mark_grid ? launch->mark_grid : (int64_t)di.cus * 8;
    const int64_t wg = launch && launch->walk_grid ? launch->walk_grid
                                                   : (int64_t)di.cus * di.walk_blocks_per_cu;
    gr.mark = (unsigned)std::max<int64_t>(1, std::min(mg, mt));
    gr.walk = (unsigned)std::max<int64_t>(1, std::min({wg, wt, (int64_t)kMaxWalkGrid}));
    gr.init = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((int64_t)di.cus * 8, (n + kBlock - 1) / kBlock));
    gr.apply = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)di.cus * di.apply_blocks_per_cu, max_items(n, m),
                              (int64_t)kMaxWalkGrid}));
    const int64_t ig = launch && launch->walk_grid ? launch->walk_grid
                                                   : (int64_t)di.cus * di.walk_ids_blocks_per_cu;
    gr.walk_ids = (unsigned)std::max<int64_t>(
        1, std::min({ig, id_groups(m) - 1, (int64_t)kMaxWalkGrid}));
    gr.ids = ids_allowed(n, m, launch);
    gr.reduce = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((int64_t)di.cus * 8, (n * 16 + kBlock - 1) / kBlock));
    return gr;
}

hipError_t launch_init(const Work& w, const dsg_csr* g, int64_t n, int64_t m, int64_t num,
                       int64_t den, int32_t max_pass, int32_t trace_cap,
                       const dsg_launch* launch, int32_t core_mode, hipStream_t s) {
    k_init_state<<<1, 64, 0, s>>>(w, g->row_ptr, n, m, num, den, max_pass,
                                  std::min(trace_cap, kTraceCap), (int32_t)part_stride(n),
                                  (int32_t)max_items(n, m),
                                  launch && (launch->flags & DSG_LAUNCH_BIN_REGIONS) ? 1 : 0,
                                  core_mode || !ids_allowed(n, m, launch)            ? 2
                                  : launch && (launch->flags & DSG_LAUNCH_ID_BUCKETS) ? 1
                                                                                     : 0,
                                  core_mode);
    return hipGetLastError();
}

// One pass of Algorithm 1 as seven launches, nine where the pass may key its
// records by neighbour id (gr.ids); `seq` numbers it for the progress word
// (when w.progress is set).  `log` brackets the kernel groups
// with events when it is on.
hipError_t enqueue_pass(const Work& w, const Grids& gr, const dsg_csr* g, int64_t n, int64_t m,
                        int32_t* best, hipStream_t s, EventLog& log, int64_t seq) {
    hipError_t e = log.begin(kKindMark);
    if (e != hipSuccess) return e;
    k_mark_count<<<gr.mark, kBlock, 0, s>>>(w, g->row_ptr, n, best);
    k_scan_tiles<<<1, kScanBlock, 0, s>>>(w, 0, n, seq);
    k_mark_scatter<<<gr.mark, kBlock, 0, s>>>(w, g->row_ptr, n, walk_tiles(m), max_bins(n));
    if ((e = hipGetLastError()) != hipSuccess || (e = log.end()) != hipSuccess ||
        (e = log.begin(kKindWalk)) != hipSuccess)
        return e;
    k_walk<<<gr.walk, kBlock, 0, s>>>(w, g->col_idx, (uint32_t)n, (uint32_t)(2 * m));
    if (gr.ids)
        k_walk_ids<<<gr.walk_ids, kBlock, 0, s>>>(w, g->col_idx, (uint32_t)n, (uint32_t)(2 * m));
    if ((e = hipGetLastError()) != hipSuccess || (e = log.end()) != hipSuccess ||
        (e = log.begin(kKindApply)) != hipSuccess)
        return e;
    k_walk_finish<<<1, kBlock, 0, s>>>(w, g->row_ptr, n, (int32_t)gr.walk, 0);
    k_apply<<<gr.apply, kApplyBlock, 0, s>>>(w);
    k_reduce<<<gr.reduce, kBlock, 0, s>>>(w);
    if (gr.ids) k_walk_finish<<<1, kBlock, 0, s>>>(w, g->row_ptr, n, (int32_t)gr.apply, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return log.end();
}

// The peel (core_mode 0) or CBDS-P (core_mode 1: k-core levels, then the
// legitimate-vertex extension, reported in *cb).
int32_t run_peel(const dsg_csr* g, int64_t n, int64_t m, int64_t eps_num, int64_t eps_den,
                 int32_t core_mode, int32_t* best_ids, int32_t* removed_at, dsg_result* out,
                 dsg_cbds_result* cb, dsg_pass_trace* trace, int32_t trace_cap,
                 const dsg_launch* launch, dsg_profile* prof, void* workspace, size_t ws_bytes,
                 void* stream) {
    if (!out || !g) return DSG_EINVAL;
    int32_t rc = check_sizes(n, m, eps_num, eps_den);
    if (rc != DSG_OK) return rc;
    if (n > 0 && !g->row_ptr) return DSG_EINVAL;
    if (m > 0 && !g->col_idx) return DSG_EINVAL;
    if (m > 0 && n < 2) return DSG_EINVAL;
    if (trace_cap < 0 || (trace_cap > 0 && !trace)) return DSG_EINVAL;
    const Layout L = layout(n, m);
    if (workspace && ws_bytes < L.total) return DSG_EINVAL;
    if (workspace && ((uintptr_t)workspace & 255u)) return DSG_EINVAL;
    if (launch && (launch->mark_grid < 0 || launch->walk_grid < 0 || launch->pass_batch < 0))
        return DSG_EINVAL;
    std::memset(out, 0, sizeof(*out));
    if (prof) std::memset(prof, 0, sizeof(*prof));
    if (cb) std::memset(cb, 0, sizeof(*cb));
    if (n == 0) return DSG_OK;

    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)workspace;
    bool owned = false;
    EventLog log;
    log.on = prof != nullptr;
    log.s = s;
    DevInfo di;
    Work w;
    int32_t max_pass, batch;
    int64_t launched = 0;
    unsigned mark_grid, walk_grid, init_grid, apply_grid, reduce_grid, walk_ids_grid;
    bool ids;

    DSG_HIP(device_info(&di));
    if (!t_host_state) {
        void* p = nullptr;
        DSG_HIP(hipHostMalloc(&p, sizeof(DevState), hipHostMallocDefault));
        t_host_state = (DevState*)p;
    }
    if (!t_progress) {
        void* p = nullptr;
        DSG_HIP(hipHostMalloc(&p, 64, hipHostMallocCoherent));
        t_progress = (int64_t*)p;
    }
    if (!base) {
        DSG_HIP(hipMalloc((void**)&base, L.total));
        owned = true;
    }
    w = make_work(base, L, removed_at);

    // core levels: every pass removes a vertex or ends a level, and every
    // level after the first removes a vertex, so 2n + 1 passes suffice
    max_pass = core_mode ? (int32_t)std::min<int64_t>(2 * n + 2, INT32_MAX)
                         : pass_bound(n, eps_num, eps_den);
    {
        const Grids gr = default_grids(di, n, m, launch);
        mark_grid = gr.mark;
        walk_grid = gr.walk;
        init_grid = gr.init;
        apply_grid = gr.apply;
        reduce_grid = gr.reduce;
        walk_ids_grid = gr.walk_ids;
        ids = gr.ids && !core_mode;
        batch = launch && launch->pass_batch ? launch->pass_batch : std::min(max_pass, 8);
    }

    DSG_HIP(log.begin(kKindInit));
    DSG_HIP(launch_init(w, g, n, m, eps_num, eps_den, max_pass, trace_cap, launch, core_mode, s));
    DSG_HIP(log.end());

    {  // the scope of pass_launches, which the error paths jump past
    // One pass, seven launches; `seq` numbers it for the progress word.
    auto pass_launches = [&](int64_t seq) -> hipError_t {
        const Grids gr{mark_grid, walk_grid, init_grid, apply_grid, reduce_grid, walk_ids_grid, ids};
        return enqueue_pass(w, gr, g, n, m, core_mode ? nullptr : best_ids, s, log, seq);
    };

    // Peeling passes run one pass ahead of the host: pass k's tile scan
    // posts whether pass k leaves survivors (and whether few), and the host
    // enqueues pass k + 1 on that, while pass k's walk and degree updates
    // still run.  No pass is then enqueued after the last one.  Core levels (many light passes,
    // grids resized between batches) and an explicit pass batch use batches
    // of passes with a host check after each; so does the rest of a peel
    // whose post did not come (the stream drained or failed first).
    const bool ahead = !core_mode && !(launch && launch->pass_batch);
    if (ahead) {
        __atomic_store_n(t_progress, (int64_t)0, __ATOMIC_RELEASE);
        w.progress = launch && (launch->flags & DSG_LAUNCH_NO_PROGRESS) ? nullptr : t_progress;
        for (int64_t seq = 1;; ++seq) {
            DSG_HIP(pass_launches(seq));
            ++launched;
            const int64_t v = wait_progress(t_progress, 4 * seq, s);
            if (v < 0 || (v & 1) || launched > (int64_t)max_pass) break;
            // survivors only decrease: after a pass with few, no later pass
            // takes walk mode 2 by itself, and its kernels need not be queued
            if ((v & 2) && !(launch && (launch->flags & DSG_LAUNCH_ID_BUCKETS))) ids = false;
        }
        w.progress = nullptr;
    }

    for (bool first = true;; first = false) {
        for (int32_t b = 0; b < batch && !(first && ahead); ++b) {
            DSG_HIP(pass_launches(0));
            ++launched;
        }
        if (best_ids && !core_mode) {
            // S~ is already in best_ids unless it is the whole graph
            DSG_HIP(log.begin(kKindExtract));
            k_extract_iota<<<init_grid, kBlock, 0, s>>>(w, n, best_ids);
            DSG_HIP(hipGetLastError());
            DSG_HIP(log.end());
        }
        DSG_HIP(hipMemcpyAsync(t_host_state, w.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
        DSG_HIP(hipStreamSynchronize(s));
        if (t_host_state->done) break;
        if (launched > (int64_t)max_pass + 1) {
            rc = DSG_EINTERNAL;
            goto done;
        }
        batch = std::min<int32_t>(batch * 2, 64);
        if (core_mode && !(launch && (launch->mark_grid || launch->walk_grid))) {
            // k-core levels run many light passes; every kernel loops over
            // its tiles with a grid stride, and the live set only shrinks,
            // so grids sized for the live set seen now stay correct and
            // dispatch far fewer idle workgroups
            const int64_t S = std::max<int64_t>(t_host_state->S, 1);
            const int64_t cap = (int64_t)di.cus * 8;
            mark_grid = (unsigned)std::max<int64_t>(1, std::min(cap, mark_tiles(S) - 1));
            walk_grid = (unsigned)std::max<int64_t>(
                1, std::min<int64_t>({(int64_t)di.cus * di.walk_blocks_per_cu,
                                      std::max<int64_t>(mark_grid, di.cus),
                                      (int64_t)kMaxWalkGrid}));
            reduce_grid = (unsigned)std::max<int64_t>(1, std::min(cap, (S * 16 + kBlock - 1) / kBlock));
        }
    }
    }  // pass_launches
    if (core_mode && t_host_state->status == kStOk) {
        // CBDS-P phase 2, then S = C_K plus the legitimate vertices; the
        // live lists and a degree array are free now and hold the flags and
        // the vertex lists
        int32_t* flag = w.list0;
        int32_t* elist = w.list1;
        int32_t* llist = w.deg0;
        // every vertex again: the grid for the whole graph, not the one the
        // level loop shrank to its last live sets
        const unsigned full = default_grids(di, n, m, launch).mark;
        DSG_HIP(log.begin(kKindExtract));
        k_cbds_eligible<<<init_grid, kBlock, 0, s>>>(w, n, flag, elist);
        k_cbds_legits<<<full, kBlock, 0, s>>>(w, g->row_ptr, g->col_idx, n, flag, elist, llist);
        k_cbds_pairs<<<full, kBlock, 0, s>>>(w, g->row_ptr, g->col_idx, n, flag, llist);
        if (best_ids) {
            k_extract_count<<<full, kBlock, 0, s>>>(w, n, flag);
            k_scan_tiles<<<1, kScanBlock, 0, s>>>(w, 1, n, 0);
            k_extract_scatter<<<full, kBlock, 0, s>>>(w, n, best_ids, flag);
        }
        DSG_HIP(hipGetLastError());
        DSG_HIP(log.end());
        DSG_HIP(hipMemcpyAsync(t_host_state, w.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
        DSG_HIP(hipStreamSynchronize(s));
    }
    {
        const DevState& h = *t_host_state;
        if (h.status == kStBadRowPtr) {
            rc = DSG_EINVAL;
            goto done;
        }
        if (h.status != kStOk) {
            rc = DSG_EINTERNAL;
            goto done;
        }
        const int64_t size = core_mode ? h.best_S + (int64_t)h.cb_nlegit : h.best_S;
        if (best_ids && h.best_count != size) {
            rc = DSG_EINTERNAL;
            goto done;
        }
        out->dens_num = h.best_E;
        out->dens_den = h.best_S;
        out->passes = h.pass;
        out->best_pass = h.best_pass;
        out->best_size = size;
        if (cb) {
            cb->core_num = h.best_E;
            cb->core_den = h.best_S;
            cb->core_k = h.best_pass + 1;
            cb->kmax = h.T;
            cb->passes = h.pass;
            cb->n_eligible = h.cb_nelig;
            cb->n_legit = h.cb_nlegit;
            cb->dens_num = h.best_E + (int64_t)h.cb_sumlegit + (int64_t)h.cb_el;
            cb->dens_den = size;
            cb->best_size = best_ids ? size : 0;
        }
        if (trace && trace_cap > 0) {
            const int32_t k = std::min(std::min(trace_cap, kTraceCap), h.pass);
            DSG_HIP(hipMemcpyAsync(trace, w.trace, sizeof(PassRecord) * (size_t)k,
                                   hipMemcpyDeviceToHost, s));
            DSG_HIP(hipStreamSynchronize(s));
        }
        if (prof) {
            prof->walked = h.tot_walked;
            prof->cross = h.tot_cross;
            prof->live_scanned = h.tot_live;
            prof->walk_list = h.tot_alist;
            for (size_t i = 0; i + 1 < log.ev.size(); i += 2) {
                float ms = 0.f;
                DSG_HIP(hipEventElapsedTime(&ms, log.ev[i], log.ev[i + 1]));
                switch (log.kind[i / 2]) {
                    case kKindInit: prof->ms_init += ms; break;
                    case kKindMark: prof->ms_mark += ms; prof->launches_mark++; break;
                    case kKindWalk: prof->ms_walk += ms; prof->launches_walk++; break;
                    case kKindApply: prof->ms_apply += ms; prof->launches_apply++; break;
                    default: prof->ms_extract += ms; break;
                }
            }
            if (log.ev.size() >= 2) {
                float ms = 0.f;
                DSG_HIP(hipEventElapsedTime(&ms, log.ev.front(), log.ev.back()));
                prof->ms_total = ms;
            }
        }
    }
done:
    if (owned) {
        // the workspace may still be in use if an error interrupted the stream
        (void)hipStreamSynchronize(s);
        (void)hipFree(base);
    }
    return rc;
}

}  // namespace

namespace dsg {

// Passes the host enqueues as kernels before the device tail takes over in
// dsg_peel_async.  A peel that needs more passes runs them in k_tail.
constexpr int32_t kAsyncHead = 16;

// dsg_peel_async (declared in host.h for the entry point that brings its own
// workspace): init, `head` passes of seven launches (each a no-op once
// the graph is empty), the device tail when the watchdog allows more passes,
// extraction and the device result.  Launch counts are fixed in advance, so
// nothing waits for the device.
int32_t peel_async(const dsg_csr* g, int64_t n, int64_t m, int64_t num, int64_t den,
                  int32_t* best_ids, int32_t* removed_at, dsg_batch_result* result,
                  const dsg_launch* launch, void* workspace, size_t ws_bytes, void* stream) {
    if (!g || !result) return DSG_EINVAL;
    const int32_t rc = check_sizes(n, m, num, den);
    if (rc != DSG_OK) return rc;
    if (n > 0 && !g->row_ptr) return DSG_EINVAL;
    if (m > 0 && !g->col_idx) return DSG_EINVAL;
    if (m > 0 && n < 2) return DSG_EINVAL;
    if (launch && (launch->mark_grid < 0 || launch->walk_grid < 0 || launch->pass_batch < 0))
        return DSG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        k_async_empty<<<1, 64, 0, s>>>(result);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? DSG_OK : map_hip(e);
    }
    const Layout L = layout(n, m);
    if (!workspace || ws_bytes < L.total || ((uintptr_t)workspace & 255u)) return DSG_EINVAL;
    DevInfo di;
    hipError_t e = device_info(&di);
    if (e != hipSuccess) return map_hip(e);
    const Work w = make_work((char*)workspace, L, removed_at);
    const Grids gr = default_grids(di, n, m, launch);
    const int32_t max_pass = pass_bound(n, num, den);
    const int32_t want = launch && launch->pass_batch ? launch->pass_batch : kAsyncHead;
    const int32_t head = std::max(1, std::min(max_pass, want));
    EventLog log;  // off
    e = launch_init(w, g, n, m, num, den, max_pass, kTraceCap, launch, 0, s);
    for (int32_t p = 0; e == hipSuccess && p < head; ++p)
        e = enqueue_pass(w, gr, g, n, m, best_ids, s, log, 0);
    if (e == hipSuccess && head < max_pass) {
        k_tail<<<1, kTailBlock, 0, s>>>(w, g->row_ptr, g->col_idx, n, 2 * m, best_ids);
        e = hipGetLastError();
    }
    if (e == hipSuccess && best_ids) {
        k_extract_iota<<<gr.init, kBlock, 0, s>>>(w, n, best_ids);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        k_async_result<<<1, 64, 0, s>>>(w, result, best_ids ? 1 : 0);
        e = hipGetLastError();
    }
    return e == hipSuccess ? DSG_OK : map_hip(e);
}

}  // namespace dsg

extern "C" {

int32_t dsg_peel_ex(const dsg_csr* g, int64_t n, int64_t m, int64_t eps_num, int64_t eps_den,
                    int32_t* best_ids, int32_t* removed_at, dsg_result* out,
                    dsg_pass_trace* trace, int32_t trace_cap, const dsg_launch* launch,
                    dsg_profile* prof, void* workspace, size_t ws_bytes, void* stream) {
    return run_peel(g, n, m, eps_num, eps_den, 0, best_ids, removed_at, out, nullptr, trace,
                    trace_cap, launch, prof, workspace, ws_bytes, stream);
}

int32_t dsg_cbds(const dsg_csr* g, int64_t n, int64_t m, int32_t* best_ids, int32_t* core,
                 dsg_cbds_result* out, dsg_pass_trace* trace, int32_t trace_cap,
                 void* workspace, size_t ws_bytes, void* stream) {
    if (!out) return DSG_EINVAL;
    dsg_result r;
    return run_peel(g, n, m, 0, 1, 1, best_ids, core, &r, out, trace, trace_cap, nullptr,
                    nullptr, workspace, ws_bytes, stream);
}

int32_t dsg_peel_async(const dsg_csr* g, int64_t n, int64_t m, int64_t eps_num,
                       int64_t eps_den, int32_t* best_ids, int32_t* removed_at,
                       dsg_batch_result* result, const dsg_launch* launch, void* workspace,
                       size_t ws_bytes, void* stream) {
    return peel_async(g, n, m, eps_num, eps_den, best_ids, removed_at, result, launch, workspace,
                      ws_bytes, stream);
}

int32_t dsg_peel(const dsg_csr* g, int64_t n, int64_t m, int64_t eps_num, int64_t eps_den,
                 int32_t* best_ids, dsg_result* out, void* workspace, size_t ws_bytes,
                 void* stream) {
    return dsg_peel_ex(g, n, m, eps_num, eps_den, best_ids, nullptr, out, nullptr, 0, nullptr,
                       nullptr, workspace, ws_bytes, stream);
}

}  // extern "C"
