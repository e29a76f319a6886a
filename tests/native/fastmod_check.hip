// Host-side check of the kernels' exact modulo (invariant-divisor magic for
// 32-bit hashes, Lemire direct remainder for 64-bit hashes) and
// bucket function against the C++ '%' operator.  Built and run by
// tests/test_fastmod.py; exits non-zero on the first mismatch.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "hg_device.h"

using namespace hg;

static bool exhaustive_u32(uint32_t d) {
    const HashParams P = make_hash_params(d, 0);
    const int T = 8;
    std::vector<int> bad(T, 0);
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t)
        th.emplace_back([&, t] {
            const uint64_t lo = (1ull << 32) / T * t, hi = (1ull << 32) / T * (t + 1);
            for (uint64_t a = lo; a < hi; ++a)
                if (mod_u32((uint32_t)a, P) != (uint32_t)(a % d)) {
                    bad[t] = 1;
                    return;
                }
        });
    for (auto& x : th) x.join();
    for (int b : bad)
        if (b) return false;
    return true;
}

int main() {
    const uint32_t full[] = {1u, 2u, 3u, 10u, 1000003u, (1u << 20), (1u << 31) - 1, 1u << 31, 4294967291u, 0xffffffffu};
    for (uint32_t d : full) {
        if (!exhaustive_u32(d)) {
            printf("FAIL u32 exhaustive d=%u\n", d);
            return 1;
        }
    }
    std::mt19937_64 rng(12345);
    std::vector<uint32_t> divs = {1u, 2u, 7u, 1u << 20, (1u << 20) + 3, 1u << 31, 0xffffffffu,
                                  0xfffffffeu, 65537u, 4096u, 4097u};
    for (int i = 0; i < 200; ++i) divs.push_back((uint32_t)(rng() | 1) >> (rng() % 31));
    for (uint32_t d : divs) {
        if (d == 0) continue;
        const HashParams p = make_hash_params(d, 0);
        const HashParams64 q = make_hash_params64(d, 0);
        for (int i = 0; i < 200000; ++i) {
            const uint32_t a = (uint32_t)rng();
            if (mod_u32(a, p) != a % d) {
                printf("FAIL u32 d=%u a=%u\n", d, a);
                return 1;
            }
            uint64_t b = rng();
            if (i % 4 == 1) b = (b / d) * d;          // multiples
            if (i % 4 == 2) b = (b / d) * d + d - 1;  // one below the next multiple
            if (i % 4 == 3) b >>= (rng() % 64);
            if (fastmod_u64(b, q.m_lo, q.m_hi, d) != (uint32_t)(b % d)) {
                printf("FAIL u64 d=%u a=%llu\n", d, (unsigned long long)b);
                return 1;
            }
        }
        const uint64_t edge[] = {0ull, 1ull, ~0ull, ~0ull - 1, 1ull << 63, (1ull << 32) - 1,
                                 1ull << 32, (uint64_t)d, (uint64_t)d - 1};
        for (uint64_t b : edge)
            if (fastmod_u64(b, q.m_lo, q.m_hi, d) != (uint32_t)(b % d)) {
                printf("FAIL u64 edge d=%u a=%llu\n", d, (unsigned long long)b);
                return 1;
            }
    }
    // the bucket function itself: fmix then modulo
    for (int i = 0; i < 1000000; ++i) {
        const uint32_t k = (uint32_t)rng(), d = (uint32_t)(rng() % 0xffffffffu) + 1;
        const uint64_t seed = rng();
        const uint32_t exp = fmix32(k ^ (uint32_t)seed) % d;
        if (KeyTraits<uint32_t>::bucket(k, make_hash_params(d, seed)) != exp) {
            printf("FAIL bucket32\n");
            return 1;
        }
        const uint64_t k64 = rng();
        if (KeyTraits<uint64_t>::bucket(k64, make_hash_params64(d, seed)) !=
            (uint32_t)(fmix64(k64 ^ seed) % d)) {
            printf("FAIL bucket64\n");
            return 1;
        }
    }
    printf("OK\n");
    return 0;
}
