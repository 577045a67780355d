// stream.hip - the measured HBM ceiling of the GPU the benchmark runs on:
// STREAM-style copy (b = a) and triad (c = a + 3 b) kernels over int32
// arrays, written for gfx950: 16-byte loads and stores, nontemporal (the
// data is touched once), four vectors in flight per thread, a grid of
// several workgroups per CU striding over the arrays.  Bytes moved per
// element: copy 8 (read 4, write 4), triad 12 (read 8, write 4).
//
// Measurement only: nothing on the peeling path calls it.
//
// Also the measured ceiling of the neighbour walk's lookups: a stream of
// uniformly random vertex ids, each read once (4 B, nontemporal), and per
// id one 8-byte gather from a table of one 8-byte word per 32 ids (the
// shape of the rank directory: live bits and a rank count), eight ids per
// thread with every id load issued before the gathers that depend on them.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace {

constexpr int kBlock = 256;
constexpr int kVec = 4;  // 16-byte vectors per thread per step

typedef int v4i __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_copy(const v4i* __restrict__ a, v4i* __restrict__ b,
                                                 int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * kBlock * kVec;
    for (int64_t i = ((int64_t)blockIdx.x * kBlock * kVec) + threadIdx.x; i < n4; i += stride) {
        v4i v[kVec];
#pragma unroll
        for (int k = 0; k < kVec; ++k) {
            const int64_t j = i + (int64_t)k * kBlock;
            if (j < n4) v[k] = __builtin_nontemporal_load(a + j);
        }
#pragma unroll
        for (int k = 0; k < kVec; ++k) {
            const int64_t j = i + (int64_t)k * kBlock;
            if (j < n4) __builtin_nontemporal_store(v[k], b + j);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_triad(const v4i* __restrict__ a,
                                                  const v4i* __restrict__ b, v4i* __restrict__ c,
                                                  int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * kBlock * kVec;
    for (int64_t i = ((int64_t)blockIdx.x * kBlock * kVec) + threadIdx.x; i < n4; i += stride) {
        v4i x[kVec], y[kVec];
#pragma unroll
        for (int k = 0; k < kVec; ++k) {
            const int64_t j = i + (int64_t)k * kBlock;
            if (j < n4) {
                x[k] = __builtin_nontemporal_load(a + j);
                y[k] = __builtin_nontemporal_load(b + j);
            }
        }
#pragma unroll
        for (int k = 0; k < kVec; ++k) {
            const int64_t j = i + (int64_t)k * kBlock;
            if (j < n4) {
                const v4i r = x[k] + 3 * y[k];
                __builtin_nontemporal_store(r, c + j);
            }
        }
    }
}

__global__ void k_fill(v4i* p, int64_t n4, int v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        p[i] = v4i{v, v + 1, v + 2, v + 3};
}

// ids: idx[i] = splitmix64(seed + i) mod 2^lg_ids (SplitMix64 finaliser,
// Steele, Lea and Flood 2014); table words: (i * 0x9E3779B1, i).
__global__ void k_gather_fill(int32_t* idx, int64_t lookups, uint2* table, int64_t words,
                              int32_t lg_ids, uint64_t seed) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < lookups; i += stride) {
        uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        idx[i] = (int32_t)(z & ((1ull << lg_ids) - 1));
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
        table[i] = make_uint2((uint32_t)i * 0x9E3779B1u, (uint32_t)i);
}

constexpr int kGatherItems = 8;

__global__ __launch_bounds__(kBlock) void k_gather(const int32_t* __restrict__ idx, int64_t lookups,
                                                   const uint2* __restrict__ table,
                                                   unsigned long long* __restrict__ sink) {
    const int64_t per = (int64_t)kBlock * kGatherItems;
    uint32_t acc = 0;
    for (int64_t base = (int64_t)blockIdx.x * per; base < lookups; base += (int64_t)gridDim.x * per) {
        int32_t x[kGatherItems];
#pragma unroll
        for (int k = 0; k < kGatherItems; ++k) {
            const int64_t j = std::min(base + (int64_t)k * kBlock + threadIdx.x, lookups - 1);
            x[k] = __builtin_nontemporal_load(idx + j);
        }
#pragma unroll
        for (int k = 0; k < kGatherItems; ++k) {
            const uint2 d = table[(uint32_t)x[k] >> 5];
            const uint32_t bit = 1u << (x[k] & 31);
            acc += d.y + __popc(d.x & (bit - 1u));
        }
    }
    // keeps the gathers live; the sum never matches
    if (acc == 0xFFFFFFFFu) atomicAdd(sink, 1ull);
}

double median(std::vector<float> v) {
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.0 : v[v.size() / 2];
}

}  // namespace

extern "C" {

// Copy and triad over arrays of `bytes` bytes each (rounded down to 16),
// `reps` timed runs of each after one untimed run, median GB/s (bytes read
// plus written per second) into *copy_gbs and *triad_gbs.  `blocks_per_cu`
// sets the grid (0: 8).  Returns 0, or the hipError_t that stopped it.
int stream_measure(size_t bytes, int reps, int blocks_per_cu, double* copy_gbs,
                   double* triad_gbs) {
    const int64_t n4 = (int64_t)(bytes / 16);
    if (n4 <= 0 || reps <= 0 || !copy_gbs || !triad_gbs) return (int)hipErrorInvalidValue;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    const unsigned grid = (unsigned)std::max(1, cus * (blocks_per_cu > 0 ? blocks_per_cu : 8));
    v4i *a = nullptr, *b = nullptr, *c = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    std::vector<float> tc, tt;
    if ((e = hipMalloc((void**)&a, (size_t)n4 * 16)) != hipSuccess) goto out;
    if ((e = hipMalloc((void**)&b, (size_t)n4 * 16)) != hipSuccess) goto out;
    if ((e = hipMalloc((void**)&c, (size_t)n4 * 16)) != hipSuccess) goto out;
    if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) goto out;
    k_fill<<<grid, kBlock>>>(a, n4, 1);
    k_fill<<<grid, kBlock>>>(b, n4, 2);
    for (int r = 0; r <= reps; ++r) {
        float ms = 0.f;
        if ((e = hipEventRecord(t0, nullptr)) != hipSuccess) goto out;
        k_copy<<<grid, kBlock>>>(a, c, n4);
        if ((e = hipEventRecord(t1, nullptr)) != hipSuccess) goto out;
        if ((e = hipEventSynchronize(t1)) != hipSuccess) goto out;
        if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) goto out;
        if (r) tc.push_back(ms);
        if ((e = hipEventRecord(t0, nullptr)) != hipSuccess) goto out;
        k_triad<<<grid, kBlock>>>(a, b, c, n4);
        if ((e = hipEventRecord(t1, nullptr)) != hipSuccess) goto out;
        if ((e = hipEventSynchronize(t1)) != hipSuccess) goto out;
        if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) goto out;
        if (r) tt.push_back(ms);
    }
    *copy_gbs = 2.0 * 16.0 * (double)n4 / (median(tc) * 1e-3) / 1e9;
    *triad_gbs = 3.0 * 16.0 * (double)n4 / (median(tt) * 1e-3) / 1e9;
out:
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(c);
    return (int)e;
}

// `lookups` random ids below 2^lg_ids (lg_ids in 5..30), one gather each
// from a table of 2^lg_ids / 32 words; `reps` timed runs after one untimed
// run, median lookups per second (in billions) into *glps.  Returns 0, or
// the hipError_t that stopped it.
int gather_measure(int64_t lookups, int32_t lg_ids, int reps, int blocks_per_cu, double* glps) {
    if (lookups <= 0 || lg_ids < 5 || lg_ids > 30 || reps <= 0 || !glps)
        return (int)hipErrorInvalidValue;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    const unsigned grid = (unsigned)std::max(1, cus * (blocks_per_cu > 0 ? blocks_per_cu : 8));
    const int64_t words = ((int64_t)1 << lg_ids) / 32;
    int32_t* idx = nullptr;
    uint2* table = nullptr;
    unsigned long long* sink = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    std::vector<float> tg;
    if ((e = hipMalloc((void**)&idx, (size_t)lookups * 4)) != hipSuccess) goto out;
    if ((e = hipMalloc((void**)&table, (size_t)words * 8)) != hipSuccess) goto out;
    if ((e = hipMalloc((void**)&sink, 8)) != hipSuccess) goto out;
    if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) goto out;
    k_gather_fill<<<grid, kBlock>>>(idx, lookups, table, words, lg_ids, 0x5DEECE66Dull);
    for (int r = 0; r <= reps; ++r) {
        float ms = 0.f;
        if ((e = hipEventRecord(t0, nullptr)) != hipSuccess) goto out;
        k_gather<<<grid, kBlock>>>(idx, lookups, table, sink);
        if ((e = hipEventRecord(t1, nullptr)) != hipSuccess) goto out;
        if ((e = hipEventSynchronize(t1)) != hipSuccess) goto out;
        if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) goto out;
        if (r) tg.push_back(ms);
    }
    *glps = (double)lookups / (median(tg) * 1e-3) / 1e9;
out:
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipFree(idx);
    (void)hipFree(table);
    (void)hipFree(sink);
    return (int)e;
}

}  // extern "C"
