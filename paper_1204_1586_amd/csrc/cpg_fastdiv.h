// Division by a run-time constant without a divide instruction: for
// 0 <= x < 2^31 and 1 <= d < 2^31,
//     floor(x / d) = (x * mul) >> shift,
// with L = ceil(log2 d), shift = 31 + L and mul = ceil(2^shift / d)
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994: an (N+1)-bit multiplier with N = 31 numerator bits).
// x * mul < 2^31 * (2^32 + 1) fits in 64 bits.  Used to unravel Khatri-Rao
// row indices into per-mode indices inside the kernels.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define CPG_HD __host__ __device__
#else
#define CPG_HD
#endif

namespace cpg {

struct FastDiv {
    uint64_t mul;
    uint32_t d;
    uint32_t shift;
};

CPG_HD inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t L = 0;
    while (L < 31 && (1ull << L) < d) ++L;
    const uint32_t shift = 31 + L;
    const uint64_t num = 1ull << shift;
    const uint64_t mul = num / d + (num % d != 0 ? 1 : 0);
    return FastDiv{mul, d, shift};
}

CPG_HD inline uint32_t fast_div(uint32_t x, const FastDiv& f) { return (uint32_t)((x * f.mul) >> f.shift); }

}  // namespace cpg
