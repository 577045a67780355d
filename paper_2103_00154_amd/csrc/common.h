// common.h - device-side state, workspace layout and wave64 helpers shared by
// the HIP translation units of libdsg.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsg {

constexpr int kBlock = 256;                      // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kMarkItems = 8;                    // live-list entries per thread
constexpr int kMarkTile = kBlock * kMarkItems;   // live-list entries per tile
constexpr int kWalkItems = 8;                    // adjacency entries per thread
constexpr int kWalkTile = kBlock * kWalkItems;   // adjacency entries per tile
constexpr int kFewRows = 4;                      // tiles over <= this many rows skip the owner table
constexpr int kMaxWalkGrid = 4096;               // walk workgroups (one partial count each)
static_assert(kWalkItems % 8 == 0, "the owner scan moves 16-byte words of 16-bit entries");
static_assert(kWalkTile < 65536, "owner indices are 16-bit");
constexpr int kTraceCap = 4096;                  // device trace records
constexpr int32_t kNever = INT32_MAX;            // removed_at of a vertex still present

// Survivor-rank bins of the degree update.  A pass's survivors are numbered
// 0..|S|-1 by their position in the compacted live list; bin b holds ranks
// [b * kBinWidth, (b + 1) * kBinWidth).  Records in a bin are 16-bit local
// ranks, and one apply workgroup keeps a whole bin's counters in LDS.
constexpr int kBinShift = 15;
constexpr int kBinWidth = 1 << kBinShift;        // 32768 ranks: 128 KB of LDS counters
constexpr int kNbLds = 1024;                     // bins the walk can stage in LDS
constexpr int kScanBlock = 256;                  // threads of the tile-scan workgroup
constexpr int kApplyBlock = 1024;                // threads of an apply workgroup
constexpr int kApplyBatch = 16;                  // record loads per lane before counting
constexpr int kApplyTiles = 4096;                // tiles whose run bounds k_apply stages in LDS
constexpr int64_t kChunkMin = 8192;              // least records per apply work item
constexpr int64_t kTargetItems = 512;            // apply work items aimed for per pass
constexpr int64_t kDirectRecords = 65536;        // at most this many records: counts applied by atomics

// Neighbour-id buckets of the degree update (walk mode 2, passes that leave
// more than kFiltBits survivors and walk at least kIdMinEntries entries).
// Bucket b holds the ids
// [b * kIdWidth, (b + 1) * kIdWidth), i.e. kIdWords consecutive rank-directory
// words.  The walk writes no survivor rank: every walked entry becomes a
// 16-bit position inside its neighbour's bucket, sorted by bucket in LDS per
// group of kIdGroupTiles walk tiles; the apply step counts the positions of
// one bucket in LDS and resolves liveness and rank from the bucket's
// directory words, staged once per work item.
constexpr int kIdShift = 15;
constexpr int kIdWidth = 1 << kIdShift;          // ids per bucket: the k_apply counters
constexpr int kIdWords = kIdWidth / 32;          // rank-directory words per bucket
constexpr int kIdMaxBuckets = 1024;              // n <= 2^25
constexpr int64_t kIdMinEntries = int64_t(1) << 25;  // least walk entries of an id-keyed pass
constexpr int kIdGroupTiles = 8;                 // walk tiles per record group
constexpr int kIdGroup = kIdGroupTiles * kWalkTile;  // adjacency entries per record group
static_assert(kIdWidth == kBinWidth, "k_apply's counters serve both kinds of bins");
static_assert(kIdGroup < 65536, "group offsets are 16-bit");

// Survivor filter of the walk: when a pass leaves at most kFiltBits
// survivors, a bitmap with the bit of hash(id) set for every survivor is
// copied into each walk workgroup's LDS, and a neighbour whose bit is clear
// skips its rank-directory gather (it cannot be a survivor).  A set bit
// proves nothing; the directory still decides.
constexpr int kFiltShift = 16;
constexpr int kFiltBits = 1 << kFiltShift;       // 65536 bits: 8 KB
constexpr int kFiltWords = kFiltBits / 32;

__device__ __host__ inline uint32_t filt_hash(uint32_t v) {
    return (v * 0x9E3779B1u) >> (32 - kFiltShift);  // Fibonacci hashing
}

// Device status codes (kept in DevState::status; mapped to dsg_status).
enum : int32_t {
    kStOk = 0,
    kStBadRowPtr = 1,    // row_ptr[0] != 0 or row_ptr[n] != 2m
    kStWatchdog = 2,     // more passes than the bound allows
    kStInvariant = 3,    // intra-pass edge count odd or negative, or E < 0
    kStExtract = 4,      // extracted set size differs from the best size
};

// Peeling state of one call, resident in the workspace.  Written by the
// init kernel and by the single thread that finishes each pass; read by
// every kernel at its start (kernel boundaries order these accesses).
struct alignas(256) DevState {
    int64_t S;          // |V| at the start of the current pass
    int64_t E;          // |E| at the start of the current pass
    int64_t best_E;     // |E(S~)| so far
    int64_t best_S;     // |S~| so far
    int64_t eps_num;
    int64_t eps_den;
    int64_t nA;         // failed vertices with degree > 0 in this pass (walk list)
    int64_t nL;         // survivors of this pass
    int64_t edges;      // adjacency entries of the walk list
    int64_t sumdeg;     // sum of the current degrees of all failed vertices
    int64_t sumdeg_surv;  // sum of the current degrees of the survivors
    unsigned long long cross;  // survivors' degree decrements (sum of the walk partials)
    int64_t best_count; // ids written by the extract kernels
    int64_t tot_walked; // statistics over all passes
    int64_t tot_cross;
    int64_t tot_live;
    int64_t tot_alist;
    int64_t chunk;      // records per apply work item in this pass
    int32_t pass;       // number of the pass being run (1-based)
    int32_t T;          // threshold of the current pass
    int32_t best_pass;
    int32_t done;       // 1 once the graph is empty or an error is recorded
    int32_t status;
    int32_t max_pass;   // watchdog bound
    int32_t trace_cap;  // records the device trace may hold
    int32_t n_tiles_walk;  // walk tiles of the current pass
    int32_t nbins;      // survivor-rank bins of the current pass
    int32_t n_items;    // apply work items of the current pass
    int32_t part_stride;  // ints per partial-count row (min(kBinWidth, n))
    int32_t max_items;  // capacity of the work-item table
    int32_t walk_mode;  // 0: records in per-tile regions, 1: records in bin regions,
                        // 2: neighbour-id positions in per-group regions
    int32_t toff_stride;  // entries per tile in the tile-offset table (bins + 1)
    int32_t force_bins;   // 1: always use bin regions (launch flag)
    int32_t apply_lanes;  // lanes that share one tile's run in k_apply (4..64)
    int32_t reduce_lanes; // lanes that share one rank in k_reduce (1..16)
    int32_t use_filt;     // 1: this pass's survivors are in the walk's survivor filter
    int32_t apply_direct; // 1: few records; k_apply decrements the degrees itself, k_reduce idles
    int32_t id_mode;      // neighbour-id buckets: 0 when they pay, 1 whenever allowed, 2 never
    int32_t id_nb;        // walk mode 2: buckets (ceil(n / kIdWidth))
    int32_t id_groups;    //   record groups of the current pass
    int32_t id_words;     //   rank-directory words (ceil(n / 32))
    uint32_t apply_next;  //   apply items taken after each workgroup's first
    // k-core levels (CBDS-P phase 1): the threshold is the level k and stays
    // there while passes remove vertices; a pass that removes none ends the
    // level, and the next level is the least degree left
    int32_t core_mode;
    int32_t min_surv;     // least degree among this pass's survivors
    int32_t jumped;       // 1: nothing failed at the level, this pass runs the next one
    uint32_t cb_nelig;    // CBDS-P phase 2: eligible outside vertices
    uint32_t cb_nlegit;   //   legitimate ones
    unsigned long long cb_sumlegit;  // their neighbours inside the core
    unsigned long long cb_el;        // edges among legitimate vertices
};

struct PassRecord {
    int64_t s_in, e_in, thresh, removed, cross, intra, walked, s_out, e_out;
};

// floor(2 (num + den) E / (S den)) capped at INT32_MAX.  The host checks
// 2(num+den)m < 2^63 and n den < 2^63, so no product overflows.
__device__ __host__ inline int32_t pass_threshold(int64_t E, int64_t S, int64_t num,
                                                  int64_t den) {
    const int64_t a = 2 * (num + den) * E;
    const int64_t b = S * den;
    const int64_t q = a / b;
    return q > (int64_t)INT32_MAX ? INT32_MAX : (int32_t)q;
}

// ---------------------------------------------------------------- wave64

__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline int wave_id() { return threadIdx.x >> 6; }

template <typename T>
__device__ inline T wave_sum(T x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

template <typename T>
__device__ inline T wave_incl_sum(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

__device__ inline int32_t wave_incl_max(int32_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x = max(x, y);
    }
    return x;
}

// Block-wide exclusive sum over NW waves; *total receives the block sum.
// `red` holds NW elements of LDS.  Contains two barriers.
template <typename T, int NW = kWaves>
__device__ inline T block_excl_sum(T x, T* red, T* total) {
    const T incl = wave_incl_sum(x);
    if (lane_id() == 63) red[wave_id()] = incl;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const T v = red[w];
        before += (w < wave_id()) ? v : T(0);
        all += v;
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

// Block-wide sum over NW waves, returned to every thread.  Two barriers.
template <typename T, int NW = kWaves>
__device__ inline T block_sum(T x, T* red) {
    x = wave_sum(x);
    if (lane_id() == 0) red[wave_id()] = x;
    __syncthreads();
    T all = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) all += red[w];
    __syncthreads();
    return all;
}

// K block-wide sums at once (every thread gets all K).  `red` holds
// K * kWaves elements of LDS.  Two barriers.
template <int K>
__device__ inline void block_sum_k(uint32_t (&x)[K], uint32_t* red) {
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = wave_sum(x[k]);
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[k * kWaves + wave_id()] = x[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        uint32_t all = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) all += red[k * kWaves + w];
        x[k] = all;
    }
    __syncthreads();
}

// K block-wide exclusive sums at once: x[k] becomes the sum over the
// threads before this one, total[k] the block sum.  `red` holds K * kWaves
// elements of LDS.  Two barriers.
template <int K>
__device__ inline void block_excl_sum_k(uint32_t (&x)[K], uint32_t* red, uint32_t (&total)[K]) {
    uint32_t incl[K];
#pragma unroll
    for (int k = 0; k < K; ++k) incl[k] = wave_incl_sum(x[k]);
    if (lane_id() == 63) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[k * kWaves + wave_id()] = incl[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t v = red[k * kWaves + w];
            before += (w < wave_id()) ? v : 0u;
            all += v;
        }
        total[k] = all;
        x[k] = before + incl[k] - x[k];
    }
    __syncthreads();
}

// Block-wide minimum of unsigned values, returned to every thread.  Two
// barriers.
template <int NW = kWaves>
__device__ inline uint32_t block_min(uint32_t x, uint32_t* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = min(x, (uint32_t)__shfl_xor(x, off, 64));
    if (lane_id() == 0) red[wave_id()] = x;
    __syncthreads();
    uint32_t all = 0xFFFFFFFFu;
#pragma unroll
    for (int w = 0; w < NW; ++w) all = min(all, red[w]);
    __syncthreads();
    return all;
}

// Block-wide exclusive max (identity `lo`).  Two barriers.
__device__ inline int32_t block_excl_max(int32_t x, int32_t* red, int32_t lo) {
    const int32_t incl = wave_incl_max(x);
    int32_t excl_in_wave = __shfl_up(incl, 1, 64);
    if (lane_id() == 0) excl_in_wave = lo;
    if (lane_id() == 63) red[wave_id()] = incl;
    __syncthreads();
    int32_t before = lo;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
        if (w < wave_id()) before = max(before, red[w]);
    __syncthreads();
    return max(before, excl_in_wave);
}

}  // namespace dsg
