// checks.h - host-side argument checks of libdsg.so that need no HIP
// runtime: the exact-integer size limits and the pass watchdog bound.  Kept
// free of HIP headers so that a plain host compiler (and its sanitizers) can
// build and test them.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dsg.h"

namespace dsg {

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Sizes and eps for which every product of the method stays inside int64:
// 2(num+den)|E| and |V| den are the two sides of the failure test, and the
// int32 CSR needs n + 1 and 2m entries.
inline int32_t check_sizes(int64_t n, int64_t m, int64_t num, int64_t den) {
    if (n < 0 || m < 0 || den < 1 || num < 0) return DSG_EINVAL;
    if (n > (int64_t)INT32_MAX - 1) return DSG_EOVERFLOW;
    if (2 * (__int128)m > (__int128)INT32_MAX) return DSG_EOVERFLOW;
    if (num > INT64_MAX - den) return DSG_EOVERFLOW;
    const __int128 lim = (__int128)1 << 63;
    if ((__int128)2 * ((__int128)num + den) * m >= lim) return DSG_EOVERFLOW;
    if ((__int128)n * den >= lim) return DSG_EOVERFLOW;
    return DSG_OK;
}

namespace detail {

// Little-endian base-2^32 natural numbers, just enough for the bound below.
using Big = std::vector<uint32_t>;

inline void big_mul(Big& a, uint64_t x) {
    unsigned __int128 carry = 0;
    for (uint32_t& limb : a) {
        const unsigned __int128 t = (unsigned __int128)limb * x + carry;
        limb = (uint32_t)t;
        carry = t >> 32;
    }
    while (carry) {
        a.push_back((uint32_t)carry);
        carry >>= 32;
    }
}

inline bool big_ge(const Big& a, const Big& b) {
    if (a.size() != b.size()) return a.size() > b.size();
    for (size_t i = a.size(); i-- > 0;)
        if (a[i] != b[i]) return a[i] > b[i];
    return true;
}

inline uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace detail

// Limb operations an exact power comparison may spend (a few ms of host
// time at most); it is needed only when the floating-point estimate below
// cannot decide.
constexpr uint64_t kPassBoundWork = uint64_t(1) << 22;

namespace detail {

// p^k >= n q^k, exactly; 0 or 1, or -1 when the limb budget would be passed.
inline int pow_ge(uint64_t p, uint64_t q, int64_t n, int64_t k) {
    Big a{1u}, b{(uint32_t)n};  // n < 2^31
    uint64_t work = 0;
    for (int64_t i = 0; i < k; ++i) {
        big_mul(a, p);
        big_mul(b, q);
        work += a.size() + b.size();
        if (work > kPassBoundWork) return -1;
    }
    return big_ge(a, b) ? 1 : 0;
}

}  // namespace detail

// Upper bound on the number of passes of a peel (the watchdog).
//
// Section 3.1: a pass that leaves survivors keeps only vertices of degree
// above 2(1+eps)|E|/|V|, and their degrees sum to at most 2|E|, so
// |S_k| (num+den) < |S_{k-1}| den.  After K passes with
// (num+den)^K >= n den^K nothing is left, so passes <= K for the least such
// K.  With eps = 0 every pass still removes a vertex, so passes <= n, and n
// caps the bound for every eps.
//
// K = ceil(ln n / ln(1+eps)).  The quotient t is computed in long double
// (64-bit mantissa: for t < 2^31 its absolute error stays near 1e-9); when t
// lies within 1e-6 of an integer k the rounding could go either way, and K
// is decided exactly instead: (num+den)^k >= n den^k in multi-limb integers (the fraction
// reduced first).  Only if that comparison would pass kPassBoundWork limb
// operations is k + 1, which is at least K, returned; *exact (optional)
// then reads false.
inline int32_t pass_bound(int64_t n, int64_t num, int64_t den, bool* exact = nullptr) {
    if (exact) *exact = true;
    if (n <= 1) return (int32_t)std::max<int64_t>(n, 0);
    if (num == 0) return (int32_t)n;
    const uint64_t g = detail::gcd64((uint64_t)num, (uint64_t)den);
    const uint64_t p = ((uint64_t)num + (uint64_t)den) / g, q = (uint64_t)den / g;
    const long double lr = log1pl((long double)(p - q) / (long double)q);
    const long double t = logl((long double)n) / lr;
    if (!(t < (long double)n)) return (int32_t)n;  // K >= n (or t not finite)
    const long double k_near = roundl(t);
    if (fabsl(t - k_near) > 1e-6L) {
        const int64_t k = std::max<int64_t>(1, (int64_t)ceill(t));
        return (int32_t)std::min<int64_t>(n, k);
    }
    const int64_t k = std::max<int64_t>(1, (int64_t)k_near);
    const int r = detail::pow_ge(p, q, n, k);
    if (r < 0) {
        if (exact) *exact = false;
        return (int32_t)std::min<int64_t>(n, k + 1);
    }
    // t > k - 1, so k - 1 passes are never enough
    return (int32_t)std::min<int64_t>(n, r ? k : k + 1);
}

}  // namespace dsg
