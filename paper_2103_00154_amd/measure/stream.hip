// stream.hip - the measured HBM ceiling of the GPU the benchmark runs on:
// STREAM-style copy (b = a) and triad (c = a + 3 b) kernels over int32
// arrays, written for gfx950: 16-byte loads and stores, nontemporal (the
// data is touched once), four vectors in flight per thread, a grid of
// several workgroups per CU striding over the arrays.  Bytes moved per
// element: copy 8 (read 4, write 4), triad 12 (read 8, write 4).
//
// Measurement only: nothing on the peeling path calls it.

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

}  // extern "C"
