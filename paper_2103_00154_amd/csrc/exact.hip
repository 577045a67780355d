// exact.hip - the exact densest subgraph on gfx950: dsg_exact_density.
//
// Section 2 names Goldberg's max-flow construction as the exact method for
// the densest subgraph, the reference point of the (2+2eps) guarantee of
// Section 3.1.  For a guess rho = p/q the network has a source s, a sink t
// and the graph's vertices; with the constant terms of Goldberg's
// capacities dropped, s->v has capacity max(0, q deg(v) - 2p), v->t has
// max(0, 2p - q deg(v)) and every edge has capacity q in both directions.
// A cut with source side {s} + S costs cut({s}) + 2(p|S| - q|E(S)|), so a
// minimum cut's source side S maximises q|E(S)| - p|S|.  Dinkelbach's
// iteration starts from the density of G and replaces the guess by the
// density of the cut side while that side is strictly denser; at the
// optimum guess the largest source side of a minimum cut is the largest
// densest subgraph (the union of all subsets of greatest density).
//
// The maximum flow is a push-relabel preflow on the device:
//
//   * the source arcs start saturated, so vertex v starts with excess
//     max(0, q deg(v) - 2p) and residual max(0, 2p - q deg(v)) towards t;
//   * a global relabel sets every height to the residual distance to t
//     (a level-synchronous search from t over reversed residual arcs; N =
//     n + 2 for vertices that cannot reach t);
//   * push launches: one wave per active vertex (excess > 0, height < N)
//     discharges it: to t while that arc has residual, then into every
//     lower neighbour, 64 arcs per step, each arc taking what the excess
//     still covers after the arcs before it (a wave prefix sum); excess
//     left after the whole row relabels the vertex to one above its lowest
//     remaining residual neighbour.  Residuals and excesses change with
//     device atomics; only a vertex's own wave lowers its excess and its
//     outgoing residuals, so concurrent waves never push more than there is
//     (the lock-free scheme of Hong and He for push-relabel on many
//     threads);
//   * global relabels alternate with batches of push launches until no
//     vertex with excess can reach t.  The preflow is then maximum, and the
//     vertices that cannot reach t form the largest minimum-cut source side.
//
// All quantities are exact int64 integers: excesses are at most 2qm <=
// 2nm < 2^62 for every graph the size checks admit.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "common.h"
#include "dsg.h"
#include "host.h"

namespace dsg {
namespace {

constexpr int kExBlock = 256;
constexpr int kExWaves = kExBlock / 64;
constexpr int kExPushLaunches = 8;  // push launches between two global relabels
constexpr int64_t kExMaxRounds = 20000;  // global relabels per flow (never reached)
constexpr int kExMaxGuesses = 4096;        // Dinkelbach steps (never reached)
constexpr int kExTile = 2048;              // vertices per tile of the set extraction

struct ExWork {
    int64_t* res;    // 2m: residual capacity of every adjacency entry's arc
    int32_t* rev;    // 2m: the entry of the reverse arc
    int64_t* ex;     // n: excess
    int64_t* rt;     // n: residual capacity towards t
    int32_t* h;      // n: height
    int32_t* tcount; // tiles + 1: members per extraction tile, then their prefix
    unsigned long long* cnt;  // 4 counters: flag / active, |S|, 2|E(S)|
};

__device__ inline int64_t ld64(const int64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int32_t ld32(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// rev[k] for every entry k = (u -> v): the position of u in v's row
// (rows are ascending; a missing reverse entry, outside the input contract,
// gets -1 and its arc is never used).
__global__ __launch_bounds__(kExBlock) void k_ex_rev(const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, int64_t n,
                                                     int32_t* __restrict__ rev) {
    const int64_t waves = (int64_t)gridDim.x * kExWaves;
    for (int64_t u = (int64_t)blockIdx.x * kExWaves + wave_id(); u < n; u += waves) {
        const int32_t r0 = rp[u], r1 = rp[u + 1];
        for (int32_t k = r0 + lane_id(); k < r1; k += 64) {
            const int32_t v = ci[k];
            int32_t found = -1;
            if ((uint64_t)(int64_t)v < (uint64_t)n) {
                int32_t lo = rp[v], hi = rp[v + 1];
                while (lo < hi) {
                    const int32_t mid = lo + ((hi - lo) >> 1);
                    const int32_t w = ci[mid];
                    if (w == (int32_t)u) {
                        found = mid;
                        break;
                    }
                    if (w < (int32_t)u) lo = mid + 1; else hi = mid;
                }
            }
            rev[k] = found;
        }
    }
}

// The preflow of guess p/q: saturated source arcs, edge residuals q.
__global__ __launch_bounds__(kExBlock) void k_ex_init(ExWork w, const int32_t* __restrict__ rp,
                                                      int64_t n, int64_t p, int64_t q) {
    const int64_t waves = (int64_t)gridDim.x * kExWaves;
    for (int64_t u = (int64_t)blockIdx.x * kExWaves + wave_id(); u < n; u += waves) {
        const int32_t r0 = rp[u], r1 = rp[u + 1];
        if (lane_id() == 0) {
            const int64_t a = q * (int64_t)(r1 - r0) - 2 * p;
            w.ex[u] = a > 0 ? a : 0;
            w.rt[u] = a < 0 ? -a : 0;
        }
        for (int32_t k = r0 + lane_id(); k < r1; k += 64) w.res[k] = w.rev[k] >= 0 ? q : 0;
    }
}

// Global relabel, level 1: vertices with a residual arc to t.
__global__ __launch_bounds__(kExBlock) void k_ex_h_init(ExWork w, int64_t n, int32_t N) {
    const int64_t stride = (int64_t)gridDim.x * kExBlock;
    for (int64_t u = (int64_t)blockIdx.x * kExBlock + threadIdx.x; u < n; u += stride)
        w.h[u] = w.rt[u] > 0 ? 1 : N;
    if (blockIdx.x == 0 && threadIdx.x == 0) w.cnt[0] = 0;
}

// Global relabel, level `lvl` -> lvl + 1: a vertex x still unlabelled with
// a residual arc x -> v into a vertex v of level lvl gets height lvl + 1.
// The arc x -> v of the entry k = (v -> x) is rev[k].
__global__ __launch_bounds__(kExBlock) void k_ex_bfs(ExWork w, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, int64_t n,
                                                     int32_t N, int32_t lvl) {
    const int64_t waves = (int64_t)gridDim.x * kExWaves;
    bool grew = false;
    for (int64_t v = (int64_t)blockIdx.x * kExWaves + wave_id(); v < n; v += waves) {
        if (w.h[v] != lvl) continue;  // uniform over the wave
        const int32_t r0 = rp[v], r1 = rp[v + 1];
        for (int32_t k = r0 + lane_id(); k < r1; k += 64) {
            const int32_t b = w.rev[k];
            if (b < 0) continue;
            const int32_t x = ci[k];
            if (w.res[b] > 0 && w.h[x] == N) {
                w.h[x] = lvl + 1;  // every writer stores the same value
                grew = true;
            }
        }
    }
    if (__ballot(grew) && lane_id() == 0) w.cnt[0] = 1;
}

// Vertices with excess that can still reach t.
__global__ __launch_bounds__(kExBlock) void k_ex_active(ExWork w, int64_t n, int32_t N) {
    const int64_t stride = (int64_t)gridDim.x * kExBlock;
    bool act = false;
    for (int64_t u = (int64_t)blockIdx.x * kExBlock + threadIdx.x; u < n; u += stride)
        act |= w.ex[u] > 0 && w.h[u] < N;
    if (__ballot(act) && lane_id() == 0) w.cnt[0] = 1;
}

// Discharge, one wave per active vertex: first to t, then through the row
// in chunks of 64 arcs.  Every arc into a lower neighbour (admissible) takes
// what the excess still covers after the admissible arcs before it (a wave
// prefix sum), so a hub pushes through 64 arcs per step.  If excess is left
// after the whole row, every admissible arc is saturated and the vertex is
// relabelled to one above its lowest remaining residual neighbour.
__global__ __launch_bounds__(kExBlock) void k_ex_push(ExWork w, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ ci, int64_t n,
                                                      int32_t N) {
    const int64_t waves = (int64_t)gridDim.x * kExWaves;
    const int lane = lane_id();
    for (int64_t u = (int64_t)blockIdx.x * kExWaves + wave_id(); u < n; u += waves) {
        // wave-uniform values are read by lane 0 and broadcast
        int64_t e = __shfl(ld64(w.ex + u), 0, 64);
        const int32_t hu = __shfl(ld32(w.h + u), 0, 64);
        if (e <= 0 || hu >= N) continue;  // uniform over the wave
        const int64_t rt = __shfl(ld64(w.rt + u), 0, 64);
        if (rt > 0) {
            // t has height 0, below every vertex
            const int64_t d = min(e, rt);
            if (lane == 0) {
                __hip_atomic_fetch_add(w.rt + u, -d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(w.ex + u, -d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            e -= d;
            if (e == 0) continue;
        }
        const int32_t r0 = rp[u], r1 = rp[u + 1];
        unsigned long long key = ~0ull;  // lowest non-admissible residual arc: h << 32 | entry
        for (int32_t c0 = r0; c0 < r1 && e > 0; c0 += 64) {
            const int32_t k = c0 + lane;
            const int64_t rk = k < r1 ? ld64(w.res + k) : 0;
            int32_t x = 0, hx = N;
            if (rk > 0) {
                x = ci[k];
                hx = ld32(w.h + x);
            }
            const bool adm = rk > 0 && hx < hu;
            if (rk > 0 && !adm) key = min(key, ((unsigned long long)(uint32_t)hx << 32) | (uint32_t)k);
            const int64_t amt = adm ? rk : 0;
            const int64_t incl = wave_incl_sum(amt);
            const int64_t tot = __shfl(incl, 63, 64);
            const int64_t before = incl - amt;
            const int64_t give = adm ? max<int64_t>(0, min(amt, e - before)) : 0;
            if (give > 0) {
                __hip_atomic_fetch_add(w.res + k, -give, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(w.res + w.rev[k], give, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(w.ex + x, give, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            const int64_t sent = min(e, tot);
            if (lane == 0 && sent > 0)
                __hip_atomic_fetch_add(w.ex + u, -sent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            e -= sent;
        }
        if (e > 0) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1)
                key = min(key, (unsigned long long)__shfl_xor(key, off, 64));
            const int32_t hn = key == ~0ull ? N : min((int32_t)(key >> 32) + 1, N);
            if (lane == 0) __hip_atomic_store(w.h + u, hn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// |S| and 2|E(S)| of the cut side S = { v : h(v) = N }, and the members per
// extraction tile.
__global__ __launch_bounds__(kExBlock) void k_ex_side(ExWork w, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ ci, int64_t n,
                                                      int32_t N) {
    __shared__ unsigned long long red[kExWaves];
    const int64_t tiles = (n + kExTile - 1) / kExTile;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        unsigned long long members = 0, twice = 0;
        for (int i = threadIdx.x; i < kExTile; i += kExBlock) {
            const int64_t v = t * kExTile + i;
            if (v < n && w.h[v] == N) {
                ++members;
                for (int32_t k = rp[v]; k < rp[v + 1]; ++k) {
                    const int32_t x = ci[k];
                    twice += (uint64_t)(int64_t)x < (uint64_t)n && w.h[x] == N;
                }
            }
        }
        members = block_sum<unsigned long long, kExWaves>(members, red);
        twice = block_sum<unsigned long long, kExWaves>(twice, red);
        if (threadIdx.x == 0) {
            w.tcount[t] = (int32_t)members;
            atomicAdd(&w.cnt[1], members);
            atomicAdd(&w.cnt[2], twice);
        }
    }
}

// Exclusive prefix of the tile counts (one workgroup).
__global__ __launch_bounds__(kExBlock) void k_ex_scan(ExWork w, int64_t tiles) {
    __shared__ int32_t red[kExWaves];
    int32_t carry = 0;
    for (int64_t c0 = 0; c0 < tiles; c0 += kExBlock) {
        const int64_t i = c0 + threadIdx.x;
        const int32_t x = i < tiles ? w.tcount[i] : 0;
        int32_t tot;
        const int32_t ex = block_excl_sum<int32_t, kExWaves>(x, red, &tot);
        if (i < tiles) w.tcount[i] = carry + ex;
        carry += tot;
    }
}

// The members of S in ascending order.
__global__ __launch_bounds__(kExBlock) void k_ex_scatter(ExWork w, int64_t n, int32_t N,
                                                         int32_t* __restrict__ out) {
    __shared__ int32_t red[kExWaves];
    const int64_t tiles = (n + kExTile - 1) / kExTile;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        int32_t pos = w.tcount[t];
        for (int c = 0; c < kExTile; c += kExBlock) {
            const int64_t v = t * kExTile + c + threadIdx.x;
            const int32_t in = v < n && w.h[v] == N ? 1 : 0;
            int32_t tot;
            const int32_t ex = block_excl_sum<int32_t, kExWaves>(in, red, &tot);
            if (in) out[pos + ex] = (int32_t)v;
            pos += tot;
        }
    }
}

struct ExLayout {
    size_t res, rev, ex, rt, h, tcount, cnt, total;
};

ExLayout ex_layout(int64_t n, int64_t m) {
    ExLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.res = take(8 * (size_t)(2 * m));
    L.rev = take(4 * (size_t)(2 * m));
    L.ex = take(8 * (size_t)n);
    L.rt = take(8 * (size_t)n);
    L.h = take(4 * (size_t)n);
    L.tcount = take(4 * (size_t)((n + kExTile - 1) / kExTile + 1));
    L.cnt = take(8 * 4);
    L.total = o;
    return L;
}

}  // namespace
}  // namespace dsg

using namespace dsg;

#define EX_HIP(expr)              \
    do {                          \
        hipError_t _e = (expr);   \
        if (_e != hipSuccess) {   \
            rc = map_hip(_e);     \
            goto done;            \
        }                         \
    } while (0)

extern "C" {

size_t dsg_exact_workspace_bytes(int64_t n, int64_t m) {
    if (check_sizes(n, m, 0, 1) != DSG_OK) return 0;
    return ex_layout(n, m).total;
}

int32_t dsg_exact_density(const dsg_csr* g, int64_t n, int64_t m, int32_t* set_ids,
                          dsg_exact_result* out, void* workspace, size_t ws_bytes,
                          void* stream) {
    if (!g || !out) return DSG_EINVAL;
    int32_t rc = check_sizes(n, m, 0, 1);
    if (rc != DSG_OK) return rc;
    if (n > 0 && !g->row_ptr) return DSG_EINVAL;
    if (m > 0 && !g->col_idx) return DSG_EINVAL;
    if (m > 0 && n < 2) return DSG_EINVAL;
    const ExLayout L = ex_layout(n, m);
    if (workspace && (ws_bytes < L.total || ((uintptr_t)workspace & 255u))) return DSG_EINVAL;
    std::memset(out, 0, sizeof(*out));
    if (n == 0) return DSG_OK;

    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)workspace;
    bool owned = false;
    ExWork w;
    const int32_t N = (int32_t)std::min<int64_t>(n + 2, INT32_MAX);
    const int64_t tiles = (n + kExTile - 1) / kExTile;
    unsigned long long hc[4] = {0, 0, 0, 0};
    int64_t e_cur = m, s_cur = n, guesses = 0, rounds_total = 0;
    int dev = 0, cus = 0;
    unsigned grid_v, grid_t;
    if (!base) {
        EX_HIP(hipMalloc((void**)&base, L.total));
        owned = true;
    }
    w.res = (int64_t*)(base + L.res);
    w.rev = (int32_t*)(base + L.rev);
    w.ex = (int64_t*)(base + L.ex);
    w.rt = (int64_t*)(base + L.rt);
    w.h = (int32_t*)(base + L.h);
    w.tcount = (int32_t*)(base + L.tcount);
    w.cnt = (unsigned long long*)(base + L.cnt);
    EX_HIP(hipGetDevice(&dev));
    EX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    grid_v = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * 16,
                                                             (n + kExWaves - 1) / kExWaves));
    grid_t = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * 8, tiles));

    k_ex_rev<<<grid_v, kExBlock, 0, s>>>(g->row_ptr, g->col_idx, n, w.rev);
    EX_HIP(hipGetLastError());

    for (;;) {
        if (++guesses > kExMaxGuesses) {
            rc = DSG_EINTERNAL;
            goto done;
        }
        // guess p / q = e_cur / s_cur in lowest terms
        int64_t a = e_cur, b = s_cur;
        while (b) {
            const int64_t t = a % b;
            a = b;
            b = t;
        }
        const int64_t p = e_cur / a, q = s_cur / a;
        k_ex_init<<<grid_v, kExBlock, 0, s>>>(w, g->row_ptr, n, p, q);
        EX_HIP(hipGetLastError());
        for (int64_t round = 0;; ++round) {
            if (round >= kExMaxRounds) {
                rc = DSG_EINTERNAL;
                goto done;
            }
            // global relabel: residual distance to t, level by level
            k_ex_h_init<<<grid_v, kExBlock, 0, s>>>(w, n, N);
            EX_HIP(hipGetLastError());
            for (int32_t lvl = 1; lvl < N; ++lvl) {
                EX_HIP(hipMemsetAsync(w.cnt, 0, 8, s));
                k_ex_bfs<<<grid_v, kExBlock, 0, s>>>(w, g->row_ptr, g->col_idx, n, N, lvl);
                EX_HIP(hipGetLastError());
                EX_HIP(hipMemcpyAsync(hc, w.cnt, 8, hipMemcpyDeviceToHost, s));
                EX_HIP(hipStreamSynchronize(s));
                if (!hc[0]) break;
            }
            EX_HIP(hipMemsetAsync(w.cnt, 0, 8, s));
            k_ex_active<<<grid_v, kExBlock, 0, s>>>(w, n, N);
            EX_HIP(hipGetLastError());
            EX_HIP(hipMemcpyAsync(hc, w.cnt, 8, hipMemcpyDeviceToHost, s));
            EX_HIP(hipStreamSynchronize(s));
            ++rounds_total;
            if (!hc[0]) break;  // maximum preflow: no excess can reach t
            for (int i = 0; i < kExPushLaunches; ++i)
                k_ex_push<<<grid_v, kExBlock, 0, s>>>(w, g->row_ptr, g->col_idx, n, N);
            EX_HIP(hipGetLastError());
        }
        // the largest minimum-cut side S: the vertices that cannot reach t
        EX_HIP(hipMemsetAsync(w.cnt, 0, 32, s));
        k_ex_side<<<grid_t, kExBlock, 0, s>>>(w, g->row_ptr, g->col_idx, n, N);
        EX_HIP(hipGetLastError());
        EX_HIP(hipMemcpyAsync(hc, w.cnt, 32, hipMemcpyDeviceToHost, s));
        EX_HIP(hipStreamSynchronize(s));
        const int64_t s_new = (int64_t)hc[1], e_new = (int64_t)(hc[2] / 2);
        if (s_new > 0 && (__int128)e_new * s_cur > (__int128)e_cur * s_new) {
            e_cur = e_new;  // strictly denser: the next guess
            s_cur = s_new;
            continue;
        }
        // the optimum guess: S is the largest densest subgraph
        if (s_new == 0 || (__int128)e_new * s_cur != (__int128)e_cur * s_new || (hc[2] & 1)) {
            rc = DSG_EINTERNAL;
            goto done;
        }
        out->dens_num = e_new;
        out->dens_den = s_new;
        out->flows = (int32_t)guesses;
        out->relabels = (int32_t)std::min<int64_t>(rounds_total, INT32_MAX);
        out->set_size = set_ids ? s_new : 0;
        if (set_ids) {
            k_ex_scan<<<1, kExBlock, 0, s>>>(w, tiles);
            k_ex_scatter<<<grid_t, kExBlock, 0, s>>>(w, n, N, set_ids);
            EX_HIP(hipGetLastError());
            EX_HIP(hipStreamSynchronize(s));
        }
        break;
    }
done:
    if (owned) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(base);
    }
    return rc;
}

}  // extern "C"
