// host_checks.cpp - drives the host-side checks of libdsg.so (csrc/checks.h)
// under a plain host compiler, so that they run with the address and
// undefined-behaviour sanitizers and can be compared with the exact bounds
// the tests compute.  Test infrastructure only.
//
// stdin: one query per line, "b n num den" (pass bound) or
// "s n m num den" (size check).  stdout: one answer per query, "b bound
// exact" or "s status".
#include <cstdio>

#include "checks.h"

int main() {
    char kind[4];
    while (std::scanf("%3s", kind) == 1) {
        if (kind[0] == 'b') {
            long long n, num, den;
            if (std::scanf("%lld %lld %lld", &n, &num, &den) != 3) return 2;
            bool exact = false;
            const int32_t k = dsg::pass_bound(n, num, den, &exact);
            std::printf("b %d %d\n", (int)k, exact ? 1 : 0);
        } else if (kind[0] == 's') {
            long long n, m, num, den;
            if (std::scanf("%lld %lld %lld %lld", &n, &m, &num, &den) != 4) return 2;
            std::printf("s %d\n", (int)dsg::check_sizes(n, m, num, den));
        } else {
            return 2;
        }
    }
    return 0;
}
