// Brute-force check of the kernels' multiply-shift division against the
// hardware divide: every divisor in [1, 4096] and a set of large ones, each
// with all numerators near multiples of d, the ends of the range and random
// samples.  Prints "ok" or the first mismatch.
#include <cstdio>
#include <cstdint>
#include <random>
#include "cpg_fastdiv.h"

static int check(uint32_t d, uint32_t x) {
    const cpg::FastDiv f = cpg::make_fastdiv(d);
    const uint32_t q = cpg::fast_div(x, f);
    if (q != x / d) {
        std::printf("mismatch d=%u x=%u got %u want %u\n", d, x, q, x / d);
        return 1;
    }
    return 0;
}

int main() {
    std::mt19937_64 g(1204);
    const uint32_t xmax = 0x7fffffffu;
    auto run = [&](uint32_t d) {
        if (check(d, 0) || check(d, xmax) || check(d, xmax - 1)) return 1;
        for (int k = 0; k < 64; ++k) {
            const uint64_t m = (uint64_t)(g() % (xmax / d + 1)) * d;
            for (int64_t o = -2; o <= 2; ++o) {
                const int64_t x = (int64_t)m + o;
                if (x >= 0 && x <= (int64_t)xmax && check(d, (uint32_t)x)) return 1;
            }
        }
        for (int k = 0; k < 64; ++k)
            if (check(d, (uint32_t)(g() % ((uint64_t)xmax + 1)))) return 1;
        return 0;
    };
    for (uint32_t d = 1; d <= 4096; ++d)
        if (run(d)) return 1;
    const uint32_t big[] = {65535, 65536, 65537, 1000003, (1u << 20) + 7, (1u << 24) - 1, (1u << 30) - 1,
                            1u << 30, (1u << 30) + 1, 0x7ffffffeu, 0x7fffffffu};
    for (uint32_t d : big)
        if (run(d)) return 1;
    for (int k = 0; k < 2000; ++k)
        if (run(1 + (uint32_t)(g() % xmax))) return 1;
    std::printf("ok\n");
    return 0;
}
