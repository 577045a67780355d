// batch.hip - many graphs peeled in one persistent launch (dsg_batch_* in
// include/dsg.h).
//
// Each workgroup is a worker: it takes the next graph from a device queue
// (graphs ordered by decreasing size, so the longest jobs start first) and
// runs every pass of Algorithm 1 (P-Bahmani, Section 3.1) for that graph on
// its own, with workgroup barriers where the paper has its global barrier.
// Per pass:
//
//   mark    part 1 over the live list: failure test deg <= T_k, ordered
//           compaction (workgroup prefix sums) of the survivors into the
//           live list (in place) and of the failures with degree > 0 into
//           the walk list, with the exclusive prefix of their row lengths
//           and, for every wave tile of the flat walk range, the walk-list
//           row that contains the tile's first entry.
//   walk    part 2: every wave walks its own tiles of the flat range of the
//           walk list's adjacency entries (hub rows split over tiles, no
//           workgroup barrier) and decrements the degree of each neighbour
//           still present; entries to vertices failing in the same pass
//           are counted (intra), so |E| drops by cross + intra / 2.
//   update  |V|, |E| and the best graph (strict improvement only).
//
// Vertex state lives in LDS as one 16-bit word per vertex for the first
// `cap` vertex ids of the graph: the degree itself while below 0xFE00, an
// index into a small LDS table of large degrees, or a marker for "failed in
// this pass", "failed earlier" and "degree kept in device memory".  Degree
// decrements are LDS atomics on the 32-bit word holding the 16-bit degree
// (a degree is at least 1 before its decrement, so no borrow crosses the
// half-word).  Vertex ids at or above `cap` (graphs larger than the LDS),
// and large degrees beyond the table, use device memory and device atomics.
//
// Batches whose largest graph has more vertices than the LDS holds 16-bit
// states use 8-bit states instead (the plan's state_bits): the degree
// itself while below 0xF0, a marker for "degree in the LDS hash table"
// (keyed by vertex id, linear probing, for the few vertices of larger
// degree), "failed in this pass", "failed earlier" and "degree kept in
// device memory" (a hash table too full to take it).  A decrement of a
// degree held in the state is an LDS atomic on its byte of the 32-bit
// word, as for 16-bit states.
//
// All arithmetic is exact integer arithmetic, so results equal those of
// dsg_peel and of a sequential peel for every launch shape.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "common.h"
#include "dsg.h"
#include "host.h"

namespace dsg {
namespace {

// 16-bit vertex states
constexpr uint32_t kStDead = 0xFFFFu;    // failed in an earlier pass
constexpr uint32_t kStNow = 0xFFFEu;     // failed in the current pass
constexpr uint32_t kStGlobal = 0xFFFDu;  // present, degree in device memory
constexpr uint32_t kStSlot0 = 0xFE00u;   // present, degree in big-degree slot s - kStSlot0
constexpr int kSlots = (int)(kStGlobal - kStSlot0);
// 8-bit vertex states
constexpr uint32_t kS8Dead = 0xFFu;      // failed in an earlier pass
constexpr uint32_t kS8Now = 0xFEu;       // failed in the current pass
constexpr uint32_t kS8Global = 0xFDu;    // present, degree in device memory
constexpr uint32_t kS8Hash = 0xF0u;      // present, degree in the LDS hash table
constexpr int kHashBits = 12;
constexpr int kHashSlots = 1 << kHashBits;  // (key, degree) pairs: 32 KB of LDS
constexpr int kHashProbes = 64;          // probes before a degree goes to device memory
constexpr int kBMarkItems = 4;           // live-list entries per thread per mark chunk
constexpr int kMinWaveTile = 64 * 4;     // smallest wave tile (sizes the tile table)
constexpr int32_t kNoStart = INT32_MIN;  // no row starts at this entry (row bases are larger)
constexpr uint64_t kPlanMagic = 0x44534742504c414eull;

// One graph of the batch, in queue order (device copy).
struct BGraph {
    int64_t rp_off, ci_off, out_off, tf_off;
    int64_t num, den;
    int32_t n, m2, max_pass, index;
};
static_assert(sizeof(BGraph) == 64, "table row");

struct alignas(256) BHead {
    uint32_t next;  // queue cursor
};

struct BWork {
    int32_t state_bits;  // 16 or 8 (the kernel instantiation this work is for)
    const BGraph* gs;
    BHead* head;
    int32_t* gdeg;  // degrees kept in device memory (ids >= cap, overflow)
    int32_t* live;  // live list (compacted in place)
    int32_t* alist; // walk list: failed vertex ids
    int32_t* apre;  // walk list: exclusive prefix of row lengths
    int32_t* abase; // walk list: row start - prefix (entry e of the flat range
                    // of a row lies at col_idx[abase + e])
    int32_t* rem;   // pass in which each vertex failed, kNever while present
    int32_t* tf;    // per wave tile: walk-list row holding its first entry
    int32_t* best;  // S~ output (may be null)
    dsg_batch_result* res;
    int32_t count;
    int32_t cap;    // vertex ids with LDS state
};

static_assert(sizeof(dsg_batch_result) == 40, "result layout");

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int32_t load_coherent(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void dec_global(int32_t* p) {
    __hip_atomic_fetch_sub(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint32_t hash_home(int32_t v) {
    return ((uint32_t)v * 0x9E3779B1u) >> (32 - kHashBits);  // Fibonacci hashing
}

// Slot of a vertex whose 8-bit state says its degree is in the hash table
// (inserted within kHashProbes probes of its home slot).
__device__ inline int32_t hash_find(const int32_t* keys, int32_t v) {
    uint32_t h = hash_home(v);
    for (int p = 0; p < kHashProbes; ++p) {
        if (keys[h] == v) return (int32_t)h;
        h = (h + 1) & (kHashSlots - 1);
    }
    return 0;  // cannot happen: the state is set only after a successful insert
}

// Degree of a vertex still present.
template <int SW>
__device__ inline int32_t live_degree(int32_t v, int32_t cap, const uint32_t* s_state,
                                      const int32_t* big, const int32_t* hkey,
                                      const int32_t* hval, const int32_t* gdeg) {
    if (v < cap) {
        if constexpr (SW == 16) {
            const uint32_t s = reinterpret_cast<const uint16_t*>(s_state)[v];
            if (s < kStSlot0) return (int32_t)s;
            if (s < kStGlobal) return big[s - kStSlot0];
        } else {
            const uint32_t s = reinterpret_cast<const uint8_t*>(s_state)[v];
            if (s < kS8Hash) return (int32_t)s;
            if (s == kS8Hash) return hval[hash_find(hkey, v)];
        }
    }
    return load_coherent(gdeg + v);
}

template <int NT, int IT, int SW>
__global__ __launch_bounds__(NT) void k_batch_peel(BWork w, const int32_t* __restrict__ rp_all,
                                                   const int32_t* __restrict__ ci_all) {
    static_assert(SW == 16 || SW == 8, "16- or 8-bit vertex states");
    constexpr int NW = NT / 64;
    constexpr int WT = 64 * IT;          // wave tile
    constexpr int CH = NT * kBMarkItems;  // mark chunk
    static_assert(IT % 4 == 0, "owner rows move as int4");
    extern __shared__ uint32_t s_state[];  // two 16-bit or four 8-bit vertex states per word
    __shared__ __align__(16) int32_t s_own[NW * WT];
    __shared__ int32_t s_big[kSlots];
    __shared__ unsigned long long s_red64[NW];
    __shared__ uint32_t s_red32[NW];
    __shared__ int32_t s_q, s_nslots;

    uint16_t* st16 = reinterpret_cast<uint16_t*>(s_state);
    uint8_t* st8 = reinterpret_cast<uint8_t*>(s_state);
    // 8-bit states: the hash table follows the states (w.cap is a multiple of 16)
    int32_t* s_hkey = reinterpret_cast<int32_t*>(s_state) + (w.cap >> 2);
    int32_t* s_hval = s_hkey + kHashSlots;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wid = wave_id();
    int32_t* own = s_own + wid * WT;

    for (;;) {
        if (tid == 0) s_q = (int32_t)atomicAdd(&w.head->next, 1u);
        __syncthreads();
        const int32_t q = s_q;
        __syncthreads();
        if (q >= w.count) break;

        const BGraph g = w.gs[q];
        const int32_t n = g.n;
        const int32_t m2 = g.m2;
        const int32_t* __restrict__ rp = rp_all + g.rp_off;
        const int32_t* __restrict__ ci = ci_all + g.ci_off;
        int32_t* __restrict__ rem = w.rem + g.out_off;
        int32_t* __restrict__ gdeg = w.gdeg + g.out_off;
        int32_t* __restrict__ live = w.live + g.out_off;
        int32_t* __restrict__ alist = w.alist + g.out_off;
        int32_t* __restrict__ apre = w.apre + g.out_off;
        int32_t* __restrict__ abase = w.abase + g.out_off;
        int32_t* __restrict__ tf = w.tf + g.tf_off;
        const int32_t cap = min(n, w.cap);

        int64_t S = n, E = m2 / 2, bE = E, bS = S;
        int32_t pass = 0, bp = 0, status = DSG_OK, found = 0;

        // the row offsets must run from 0 to 2m; that they never decrease
        // is checked by the first mark, chunk by chunk, before any use
        if (n > 0 && (rp[0] != 0 || rp[n] != m2)) status = DSG_EINVAL;
        if (tid == 0) s_nslots = 0;
        if constexpr (SW == 8)
            for (int i = tid; i < kHashSlots; i += NT) s_hkey[i] = -1;
        __syncthreads();

        while (status == DSG_OK && S > 0) {
            ++pass;
            if (pass > g.max_pass) {
                status = DSG_EINTERNAL;
                break;
            }
            const int32_t T = pass_threshold(E, S, g.num, g.den);
            const int32_t nlive = (int32_t)S;

            // ------------------------------------------------ mark
            int32_t nA = 0, nL = 0, W = 0;
            for (int32_t base = 0; base < nlive; base += CH) {
                int32_t v[kBMarkItems], d[kBMarkItems], rs[kBMarkItems], rl[kBMarkItems];
                const int32_t i0 = base + tid * kBMarkItems;
                // loads first (clamped indices, no load inside a branch)
                if (pass == 1) {
                    int32_t re[kBMarkItems];
#pragma unroll
                    for (int j = 0; j < kBMarkItems; ++j) {
                        const int32_t i = min(i0 + j, nlive - 1);
                        rs[j] = rp[i];
                        re[j] = rp[i + 1];
                    }
                    // with row_ptr[0] = 0, a row that ends beyond 2m or
                    // before it starts is the first sign of bad offsets;
                    // rows before it are valid, so nothing was misused yet
                    int32_t bad = 0;
#pragma unroll
                    for (int j = 0; j < kBMarkItems; ++j) {
                        const bool ok = i0 + j < nlive;
                        v[j] = ok ? i0 + j : -1;
                        rl[j] = re[j] - rs[j];
                        d[j] = rl[j];
                        if (ok && (rl[j] < 0 || re[j] > m2)) bad = 1;
                    }
                    if (__syncthreads_or(bad)) {
                        status = DSG_EINVAL;
                        break;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < kBMarkItems; ++j) v[j] = live[min(i0 + j, nlive - 1)];
#pragma unroll
                    for (int j = 0; j < kBMarkItems; ++j) {
                        if (i0 + j >= nlive) v[j] = -1;
                        d[j] = v[j] >= 0 ? live_degree<SW>(v[j], cap, s_state, s_big, s_hkey,
                                                           s_hval, gdeg)
                                         : 0;
                    }
                    int32_t re[kBMarkItems];
#pragma unroll
                    for (int j = 0; j < kBMarkItems; ++j) {
                        // row bounds of the failures (a harmless row 0 otherwise)
                        const int32_t x = (v[j] >= 0 && d[j] > 0 && d[j] <= T) ? v[j] : 0;
                        rs[j] = rp[x];
                        re[j] = rp[x + 1];
                    }
#pragma unroll
                    for (int j = 0; j < kBMarkItems; ++j) rl[j] = re[j] - rs[j];
                }
                uint32_t cA = 0, cL = 0, sl = 0;
#pragma unroll
                for (int j = 0; j < kBMarkItems; ++j) {
                    if (v[j] < 0) continue;
                    if (d[j] > T) {
                        ++cL;
                    } else if (d[j] > 0) {
                        ++cA;
                        sl += (uint32_t)rl[j];
                    }
                }
                // one scan for the three counts: row-length sum (< 2^31 for a
                // valid CSR) in the low word, walk-list and live-list counts
                // (<= CH < 2^16) in the two high half-words
                const unsigned long long mine = (unsigned long long)sl |
                                                ((unsigned long long)cA << 32) |
                                                ((unsigned long long)cL << 48);
                unsigned long long tot;
                const unsigned long long ex =
                    block_excl_sum<unsigned long long, NW>(mine, s_red64, &tot);
                int32_t oa = nA + (int32_t)((ex >> 32) & 0xFFFFu);
                int32_t ol = nL + (int32_t)(ex >> 48);
                int32_t wo = W + (int32_t)(uint32_t)ex;
#pragma unroll
                for (int j = 0; j < kBMarkItems; ++j) {
                    const int32_t x = v[j];
                    if (x < 0) continue;
                    if (d[j] > T) {
                        live[ol++] = x;
                        if (pass == 1) {
                            rem[x] = kNever;
                            const int32_t dx = d[j];
                            bool in_lds = false;
                            if (x < cap) {
                                if constexpr (SW == 16) {
                                    if (dx < (int32_t)kStSlot0) {
                                        st16[x] = (uint16_t)dx;
                                        in_lds = true;
                                    } else {
                                        const int32_t s = atomicAdd(&s_nslots, 1);
                                        if (s < kSlots) {
                                            s_big[s] = dx;
                                            st16[x] = (uint16_t)(kStSlot0 + s);
                                            in_lds = true;
                                        } else {
                                            st16[x] = (uint16_t)kStGlobal;
                                        }
                                    }
                                } else {
                                    if (dx < (int32_t)kS8Hash) {
                                        st8[x] = (uint8_t)dx;
                                        in_lds = true;
                                    } else {
                                        // linear probing from the home slot
                                        uint32_t h = hash_home(x);
                                        for (int p = 0; p < kHashProbes; ++p) {
                                            if (atomicCAS(&s_hkey[h], -1, x) == -1) {
                                                s_hval[h] = dx;
                                                in_lds = true;
                                                break;
                                            }
                                            h = (h + 1) & (kHashSlots - 1);
                                        }
                                        st8[x] = (uint8_t)(in_lds ? kS8Hash : kS8Global);
                                        if (!in_lds) atomicAdd(&s_nslots, 1);
                                    }
                                }
                            }
                            if (!in_lds) gdeg[x] = dx;
                        }
                    } else {
                        rem[x] = pass;
                        if (x < cap) {
                            if constexpr (SW == 16)
                                st16[x] = (uint16_t)(d[j] > 0 ? kStNow : kStDead);
                            else
                                st8[x] = (uint8_t)(d[j] > 0 ? kS8Now : kS8Dead);
                        }
                        if (d[j] > 0) {
                            alist[oa] = x;
                            apre[oa] = wo;
                            abase[oa] = rs[j] - wo;
                            // wave tiles whose first entry lies in this row
                            const int32_t end = wo + rl[j];
                            for (int32_t t = (wo + WT - 1) / WT; t * WT < end; ++t) tf[t] = oa;
                            ++oa;
                            wo = end;
                        }
                    }
                }
                nA += (int32_t)((tot >> 32) & 0xFFFFu);
                nL += (int32_t)(tot >> 48);
                W += (int32_t)(uint32_t)tot;
            }
            if (status != DSG_OK) break;
            __syncthreads();
            // degrees in device memory are updated with device atomics and
            // read with L1-bypassing loads: order them at device scope.
            // Graphs whose state is all in LDS need only the barrier (one
            // workgroup owns a graph, and its plain stores and loads meet
            // in the CU's own cache).  The slot count is final after pass 1.
            const bool dev_state = n > cap || s_nslots > (SW == 16 ? kSlots : 0);
            if (dev_state) {
                __threadfence();
                __syncthreads();
            }

            // ------------------------------------------------ walk
            uint32_t cross = 0, intra = 0, badc = 0;
            if (nL > 0 && W > 0) {
                const int32_t ntile = (W + WT - 1) / WT;
                // software pipeline: the row holding a tile's first entry, its
                // base, and the starts and bases of the 256 rows after it are
                // loaded one tile ahead, while the wave works on the previous
                // tile
                int32_t rc = wid < ntile ? tf[wid] : 0;
                int32_t bc = abase[rc];
                int32_t pst[4], pab[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int32_t r = min(rc + 1 + 64 * k + lane, nA - 1);
                    pst[k] = apre[r];
                    pab[k] = abase[r];
                }
                for (int32_t t = wid; t < ntile; t += NW) {
                    const int32_t t0 = t * WT;
                    const int32_t len = min(WT, W - t0);
                    const int32_t tn = t + NW;
                    const int32_t rcn = tn < ntile ? tf[tn] : 0;
                    // the base of the row starting at each entry, kNoStart
                    // elsewhere (256 rows per step, loads first)
                    {
                        int4* o4 = reinterpret_cast<int4*>(own + lane * IT);
#pragma unroll
                        for (int k = 0; k < IT / 4; ++k)
                            o4[k] = make_int4(kNoStart, kNoStart, kNoStart, kNoStart);
                    }
                    wave_sync();
                    for (int32_t r0 = rc + 1; r0 < nA; r0 += 256) {
                        int32_t st[4], sb[4];
                        if (r0 == rc + 1) {
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                st[k] = pst[k];
                                sb[k] = pab[k];
                            }
                        } else {
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                const int32_t r = min(r0 + 64 * k + lane, nA - 1);
                                st[k] = apre[r];
                                sb[k] = abase[r];
                            }
                        }
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int32_t r = r0 + 64 * k + lane;
                            if (r < nA && st[k] < t0 + len) own[st[k] - t0] = sb[k];
                        }
                        // rows start in increasing order: stop once the last
                        // row of this step lies beyond the tile
                        if (__shfl(st[3], 63, 64) >= t0 + len) break;
                    }
                    wave_sync();
                    // base of every entry: the last row start at or before it
                    // (forward fill; the tile's first row, rc, starts before
                    // the tile and has base bc)
                    {
                        int4* o4 = reinterpret_cast<int4*>(own + lane * IT);
                        int32_t bv[IT];
#pragma unroll
                        for (int k = 0; k < IT / 4; ++k) {
                            const int4 x = o4[k];
                            bv[4 * k + 0] = x.x;
                            bv[4 * k + 1] = x.y;
                            bv[4 * k + 2] = x.z;
                            bv[4 * k + 3] = x.w;
                        }
                        int32_t last = kNoStart;
#pragma unroll
                        for (int i = 0; i < IT; ++i) last = bv[i] != kNoStart ? bv[i] : last;
                        // the last start of the lanes before this one
                        int32_t carry = last;
#pragma unroll
                        for (int off = 1; off < 64; off <<= 1) {
                            const int32_t y = __shfl_up(carry, off, 64);
                            if (lane >= off && carry == kNoStart) carry = y;
                        }
                        carry = __shfl_up(carry, 1, 64);
                        if (lane == 0 || carry == kNoStart) carry = bc;
#pragma unroll
                        for (int i = 0; i < IT; ++i) {
                            if (bv[i] == kNoStart) bv[i] = carry;
                            carry = bv[i];
                        }
                        wave_sync();
#pragma unroll
                        for (int k = 0; k < IT / 4; ++k)
                            o4[k] = make_int4(bv[4 * k + 0], bv[4 * k + 1], bv[4 * k + 2],
                                              bv[4 * k + 3]);
                    }
                    wave_sync();
                    // neighbour ids, consecutive lanes on consecutive
                    // entries.  Every stage issues all of its loads before
                    // the next stage needs them (no load inside a branch):
                    // lanes past the tile end re-read its last entry.
                    int32_t u[IT];
                    {
                        int32_t ab[IT];
#pragma unroll
                        for (int j = 0; j < IT; ++j) ab[j] = own[min(j * 64 + lane, len - 1)];
#pragma unroll
                        for (int j = 0; j < IT; ++j)
                            u[j] = __builtin_nontemporal_load(ci + ab[j] + t0 +
                                                              min(j * 64 + lane, len - 1));
                    }
                    // next tile's row starts, in flight during this tile's
                    // state lookups and decrements
                    bc = abase[rcn];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int32_t r = min(rcn + 1 + 64 * k + lane, nA - 1);
                        pst[k] = apre[r];
                        pab[k] = abase[r];
                    }
                    // states: the LDS word for ids below cap, the removal
                    // pass (device memory) above
                    uint32_t sv[IT];
#pragma unroll
                    for (int j = 0; j < IT; ++j) {
                        const int32_t x = u[j];
                        const bool in = (uint32_t)x < (uint32_t)cap;
                        if constexpr (SW == 16) {
                            const uint32_t st = st16[in ? x : 0];
                            sv[j] = in ? st : kStDead;
                        } else {
                            const uint32_t st = st8[in ? x : 0];
                            sv[j] = in ? st : kS8Dead;
                        }
                    }
                    int32_t rv[IT];
#pragma unroll
                    for (int j = 0; j < IT; ++j) rv[j] = 0;
                    if (n > cap) {
#pragma unroll
                        for (int j = 0; j < IT; ++j) {
                            const int32_t x = u[j];
                            rv[j] = rem[(x >= cap && x < n) ? x : 0];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < IT; ++j) {
                        const int32_t x = u[j];
                        if (j * 64 + lane >= len) continue;
                        if ((uint32_t)x >= (uint32_t)n) {
                            ++badc;
                        } else if (x < cap) {
                            const uint32_t st = sv[j];
                            if constexpr (SW == 16) {
                                if (st < kStSlot0) {
                                    atomicSub(&s_state[x >> 1], 1u << ((x & 1) << 4));
                                    ++cross;
                                } else if (st < kStGlobal) {
                                    atomicSub(&s_big[st - kStSlot0], 1);
                                    ++cross;
                                } else if (st == kStGlobal) {
                                    dec_global(gdeg + x);
                                    ++cross;
                                } else if (st == kStNow) {
                                    ++intra;
                                }
                            } else {
                                // a degree is >= 1 before its decrement, so no
                                // borrow crosses its byte
                                if (st < kS8Hash) {
                                    atomicSub(&s_state[x >> 2], 1u << ((x & 3) << 3));
                                    ++cross;
                                } else if (st == kS8Hash) {
                                    atomicSub(&s_hval[hash_find(s_hkey, x)], 1);
                                    ++cross;
                                } else if (st == kS8Global) {
                                    dec_global(gdeg + x);
                                    ++cross;
                                } else if (st == kS8Now) {
                                    ++intra;
                                }
                            }
                        } else if (rv[j] == kNever) {
                            dec_global(gdeg + x);
                            ++cross;
                        } else if (rv[j] == pass) {
                            ++intra;
                        }
                    }
                    rc = rcn;
                }
            }
            if (dev_state) __threadfence();
            const unsigned long long ci_sum = block_sum<unsigned long long, NW>(
                (unsigned long long)cross | ((unsigned long long)intra << 32), s_red64);
            const uint32_t bad_sum = block_sum<uint32_t, NW>(badc, s_red32);

            // ------------------------------------------------ update
            const int64_t cr = (int64_t)(ci_sum & 0xFFFFFFFFull);
            const int64_t in = (int64_t)(ci_sum >> 32);
            if (bad_sum) {
                status = DSG_EINVAL;
                break;
            }
            const int64_t Eo = nL > 0 ? E - cr - in / 2 : 0;
            if ((nL > 0 && (in & 1)) || Eo < 0) {
                status = DSG_EINTERNAL;
                break;
            }
            S = nL;
            E = Eo;
            if (S > 0 && E * bS > bE * S) {
                bE = E;
                bS = S;
                bp = pass;
            }
            // this pass's failures are gone from the next pass on
            for (int32_t r = tid; r < nA; r += 4 * NT) {
                int32_t x[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) x[k] = alist[min(r + k * NT, nA - 1)];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (r + k * NT < nA && x[k] < cap) {
                        if constexpr (SW == 16)
                            st16[x[k]] = (uint16_t)kStDead;
                        else
                            st8[x[k]] = (uint8_t)kS8Dead;
                    }
            }
        }

        // ---------------------------------------------------- extract
        if (status == DSG_OK && w.best && n > 0) {
            int32_t* __restrict__ out = w.best + g.out_off;
            for (int32_t base = 0; base < n; base += CH) {
                const int32_t i0 = base + tid * kBMarkItems;
                uint32_t keep = 0, c = 0;
                int32_t ra[kBMarkItems];
#pragma unroll
                for (int j = 0; j < kBMarkItems; ++j) ra[j] = rem[min(i0 + j, n - 1)];
#pragma unroll
                for (int j = 0; j < kBMarkItems; ++j) {
                    if (i0 + j < n && ra[j] > bp) {
                        keep |= 1u << j;
                        ++c;
                    }
                }
                uint32_t tot;
                uint32_t at = block_excl_sum<uint32_t, NW>(c, s_red32, &tot);
                at += (uint32_t)found;
#pragma unroll
                for (int j = 0; j < kBMarkItems; ++j)
                    if (keep >> j & 1u) out[at++] = i0 + j;
                found += (int32_t)tot;
            }
            if (found != bS) status = DSG_EINTERNAL;
        }
        if (tid == 0) {
            dsg_batch_result r;
            r.dens_num = n > 0 ? bE : 0;
            r.dens_den = n > 0 ? bS : 0;
            r.passes = pass;
            r.best_pass = bp;
            r.best_size = found;
            r.status = status;
            r.reserved = 0;
            w.res[g.index] = r;
        }
        __syncthreads();
    }
}

__global__ void k_batch_reset(BHead* head) {
    if (threadIdx.x == 0) head->next = 0;
}

// ------------------------------------------------------------------ host

template <int NT, int IT, int SW>
hipError_t launch_one(const dsg_batch_plan* p, const BWork& w, const int32_t* rp,
                      const int32_t* ci, hipStream_t s) {
    hipLaunchKernelGGL((k_batch_peel<NT, IT, SW>), dim3(p->grid), dim3(NT), (size_t)p->lds_bytes,
                       s, w, rp, ci);
    return hipGetLastError();
}

template <int NT, int IT, int SW>
const void* kernel_ptr() {
    return reinterpret_cast<const void*>(&k_batch_peel<NT, IT, SW>);
}

// Supported (block, walk_items) shapes (1024 x 16 would spill registers),
// each with 16- and 8-bit vertex states.
const void* batch_kernel(int block, int items, int bits) {
#define DSG_SHAPE(NT, IT)                                   \
    if (block == NT && items == IT)                         \
        return bits == 8 ? kernel_ptr<NT, IT, 8>() : kernel_ptr<NT, IT, 16>();
    DSG_SHAPE(256, 4) DSG_SHAPE(256, 8) DSG_SHAPE(256, 16)
    DSG_SHAPE(512, 4) DSG_SHAPE(512, 8) DSG_SHAPE(512, 16)
    DSG_SHAPE(1024, 4) DSG_SHAPE(1024, 8)
#undef DSG_SHAPE
    return nullptr;
}

hipError_t batch_launch(const dsg_batch_plan* p, const BWork& w, const int32_t* rp,
                        const int32_t* ci, hipStream_t s) {
#define DSG_SHAPE(NT, IT)                                            \
    if (p->block == NT && p->walk_items == IT)                       \
        return p->state_bits == 8 ? launch_one<NT, IT, 8>(p, w, rp, ci, s) \
                                  : launch_one<NT, IT, 16>(p, w, rp, ci, s);
    DSG_SHAPE(256, 4) DSG_SHAPE(256, 8) DSG_SHAPE(256, 16)
    DSG_SHAPE(512, 4) DSG_SHAPE(512, 8) DSG_SHAPE(512, 16)
    DSG_SHAPE(1024, 4) DSG_SHAPE(1024, 8)
#undef DSG_SHAPE
    return hipErrorInvalidValue;
}

struct BLayout {
    size_t head, table, tf, gdeg, live, alist, apre, abase, rem, total;
};

BLayout batch_layout(int64_t count, int64_t entries, int64_t out_len) {
    BLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.head = take(sizeof(BHead));
    L.table = take(sizeof(BGraph) * (size_t)count);
    L.tf = take(4 * (size_t)(entries / kMinWaveTile + 2 * count + 1));
    L.gdeg = take(4 * (size_t)out_len);
    L.live = take(4 * (size_t)out_len);
    L.alist = take(4 * (size_t)out_len);
    L.apre = take(4 * (size_t)out_len);
    L.abase = take(4 * (size_t)out_len);
    L.rem = take(4 * (size_t)out_len);
    L.total = o;
    return L;
}

struct BDevInfo {
    int cus = 0;
    int lds_per_cu = 0;
    int lds_per_block = 0;
    bool ready = false;
};
std::mutex g_bmu;
BDevInfo g_binfo[64];

hipError_t batch_device_info(BDevInfo* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_bmu);
    BDevInfo& d = g_binfo[dev];
    if (!d.ready) {
        e = hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&d.lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                  dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&d.lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) return e;
        if (d.lds_per_cu <= 0) d.lds_per_cu = d.lds_per_block;
        d.ready = true;
    }
    *out = d;
    return hipSuccess;
}

}  // namespace
}  // namespace dsg

using namespace dsg;

extern "C" {

size_t dsg_batch_workspace_bytes(int32_t count, int64_t entries, int64_t out_len) {
    if (count < 0 || entries < 0 || out_len < 0) return 0;
    if (out_len > ((int64_t)1 << 40) || entries > ((int64_t)1 << 42)) return 0;
    return batch_layout(count, entries, out_len).total;
}

int32_t dsg_batch_prepare(const dsg_batch_graph* graphs, int32_t count, int64_t row_ptr_len,
                          int64_t col_idx_len, int64_t out_len, const dsg_batch_launch* launch,
                          void* workspace, size_t ws_bytes, void* stream, dsg_batch_plan* plan) {
    if (!plan || count < 0 || (count > 0 && !graphs)) return DSG_EINVAL;
    if (row_ptr_len < 0 || col_idx_len < 0 || out_len < 0) return DSG_EINVAL;
    if (!workspace || ((uintptr_t)workspace & 255u)) return DSG_EINVAL;

    int32_t block = 512, bpc = 1, items = 8, grid = 0;
    if (launch) {
        if (launch->block) block = launch->block;
        if (launch->blocks_per_cu) bpc = launch->blocks_per_cu;
        if (launch->walk_items) items = launch->walk_items;
        grid = launch->grid;
    }
    if (bpc < 1 || bpc > 8 || grid < 0 || !batch_kernel(block, items, 16)) return DSG_EINVAL;

    // per-graph checks, the device table and the queue order
    std::vector<BGraph> tab((size_t)count);
    std::vector<std::pair<int64_t, int64_t>> outs;
    outs.reserve((size_t)count);
    int64_t tf_at = 0, entries = 0, nmax = 0;
    for (int32_t i = 0; i < count; ++i) {
        const dsg_batch_graph& g = graphs[i];
        if (g.reserved != 0) return DSG_EINVAL;
        const int32_t rc = check_sizes(g.n, g.m, g.eps_num, g.eps_den);
        if (rc != DSG_OK) return rc;
        if (g.row_ptr_off < 0 || g.col_idx_off < 0 || g.out_off < 0) return DSG_EINVAL;
        // an empty graph reads no row offsets
        if (g.row_ptr_off > row_ptr_len || (g.n > 0 && g.row_ptr_off > row_ptr_len - (g.n + 1)))
            return DSG_EINVAL;
        if (g.col_idx_off > col_idx_len - 2 * g.m) return DSG_EINVAL;
        if (g.out_off > out_len - g.n) return DSG_EINVAL;
        if (g.n > 0) outs.emplace_back(g.out_off, g.n);
        BGraph& b = tab[(size_t)i];
        b.rp_off = g.row_ptr_off;
        b.ci_off = g.col_idx_off;
        b.out_off = g.out_off;
        b.tf_off = tf_at;
        tf_at += 2 * g.m / kMinWaveTile + 2;
        entries += 2 * g.m;
        b.num = g.eps_num;
        b.den = g.eps_den;
        b.n = (int32_t)g.n;
        nmax = std::max<int64_t>(nmax, g.n);
        b.m2 = (int32_t)(2 * g.m);
        b.max_pass = pass_bound(g.n, g.eps_num, g.eps_den);
        b.index = i;
    }
    const size_t need = dsg_batch_workspace_bytes(count, entries, out_len);
    if (need == 0 || ws_bytes < need) return DSG_EINVAL;
    std::sort(outs.begin(), outs.end());
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i - 1].first + outs[i - 1].second > outs[i].first) return DSG_EINVAL;
    // largest graphs first: adjacency entries, then vertices, then table order
    std::stable_sort(tab.begin(), tab.end(), [](const BGraph& a, const BGraph& b) {
        const int64_t wa = (int64_t)a.m2 + a.n, wb = (int64_t)b.m2 + b.n;
        return wa > wb;
    });

    BDevInfo di;
    hipError_t e = batch_device_info(&di);
    if (e != hipSuccess) return map_hip(e);
    // LDS per workgroup left after the kernel's static tables, for the
    // vertex states of each state width
    const int64_t budget = std::min<int64_t>(di.lds_per_block, di.lds_per_cu / bpc);
    int64_t dyn_w[2] = {0, 0};  // 16-bit, 8-bit
    for (int k = 0; k < 2; ++k) {
        const void* fn = batch_kernel(block, items, k ? 8 : 16);
        hipFuncAttributes attr;
        e = hipFuncGetAttributes(&attr, fn);
        if (e != hipSuccess) return map_hip(e);
        dyn_w[k] = ((budget - (int64_t)attr.sharedSizeBytes) / 4) * 4;
        // allow the largest request any plan of this kernel can make
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(di.lds_per_block - (int64_t)attr.sharedSizeBytes));
        if (e != hipSuccess) return map_hip(e);
    }
    if (dyn_w[0] < 4) return DSG_EINVAL;
    // 16-bit states unless the largest graph needs more vertices than they
    // hold and 8-bit states (one byte per vertex after a 32 KB hash table of
    // large degrees) hold more
    const int64_t cap16 = 2 * (dyn_w[0] / 4);
    const int64_t cap8 = std::max<int64_t>(0, (dyn_w[1] - 8 * (int64_t)kHashSlots) & ~(int64_t)15);
    const bool use8 = nmax > cap16 && cap8 > cap16;
    const int64_t dyn = use8 ? dyn_w[1] : dyn_w[0];

    const BLayout L = batch_layout(count, entries, out_len);
    char* base = static_cast<char*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (count > 0) {
        e = hipMemcpyAsync(base + L.table, tab.data(), sizeof(BGraph) * tab.size(),
                           hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return map_hip(e);
    }

    std::memset(plan, 0, sizeof(*plan));
    plan->count = count;
    plan->block = block;
    plan->blocks_per_cu = bpc;
    plan->walk_items = items;
    const int64_t g_def = (int64_t)di.cus * bpc;
    plan->grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>(grid ? grid : g_def, count));
    plan->lds_bytes = (int32_t)dyn;
    plan->lds_vertices = (int32_t)std::min<int64_t>(use8 ? cap8 : cap16, INT32_MAX);
    plan->state_bits = use8 ? 8 : 16;
    plan->out_len = out_len;
    plan->workspace = workspace;
    plan->ws_bytes = need;
    plan->reserved[0] = (int64_t)kPlanMagic;
    plan->reserved[1] = entries;
    return DSG_OK;
}

int32_t dsg_batch_run(const dsg_batch_plan* plan, const int32_t* row_ptr, const int32_t* col_idx,
                      int32_t* best_ids, int32_t* removed_at, dsg_batch_result* results,
                      void* stream) {
    if (!plan || plan->reserved[0] != (int64_t)kPlanMagic || !plan->workspace) return DSG_EINVAL;
    if (plan->count == 0) return DSG_OK;
    if (!results || !row_ptr || !col_idx) return DSG_EINVAL;
    const BLayout L = batch_layout(plan->count, plan->reserved[1], plan->out_len);
    char* base = static_cast<char*>(plan->workspace);
    BWork w;
    w.gs = reinterpret_cast<const BGraph*>(base + L.table);
    w.head = reinterpret_cast<BHead*>(base + L.head);
    w.gdeg = reinterpret_cast<int32_t*>(base + L.gdeg);
    w.live = reinterpret_cast<int32_t*>(base + L.live);
    w.alist = reinterpret_cast<int32_t*>(base + L.alist);
    w.apre = reinterpret_cast<int32_t*>(base + L.apre);
    w.abase = reinterpret_cast<int32_t*>(base + L.abase);
    w.rem = removed_at ? removed_at : reinterpret_cast<int32_t*>(base + L.rem);
    w.tf = reinterpret_cast<int32_t*>(base + L.tf);
    w.best = best_ids;
    w.res = results;
    w.count = plan->count;
    w.cap = plan->lds_vertices;
    w.state_bits = plan->state_bits;
    if (w.state_bits != 16 && w.state_bits != 8) return DSG_EINVAL;
    if (w.state_bits == 8 &&
        (w.cap < 0 || (w.cap & 15) || (int64_t)w.cap + 8 * (int64_t)kHashSlots > plan->lds_bytes))
        return DSG_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    k_batch_reset<<<1, 64, 0, s>>>(w.head);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = batch_launch(plan, w, row_ptr, col_idx, s);
    return e == hipSuccess ? DSG_OK : map_hip(e);
}

}  // extern "C"
