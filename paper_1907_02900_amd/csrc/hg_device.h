// Device-side building blocks shared by the HashGraph kernels (gfx950, wave64).
//
//  * the hash of Eq. 1: MurmurHash3 finalisers fmix32 / fmix64 followed by an
//    exact modulo by V.  32-bit hashes divide by the invariant V with a
//    multiply-high and a shift (Granlund & Montgomery 1994), 64-bit hashes
//    use Lemire's direct remainder (Lemire, Kaser, Kurz, "Faster Remainder by
//    Direct Computation", 2019): for a < 2^64 and d < 2^32,
//    M = ceil(2^128 / d) gives a mod d = floor(((M * a) mod 2^128) * d / 2^128).
//  * wave64 helpers: lane id, masked popcount below the lane (mbcnt), ballots,
//    wave and block exclusive scans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

constexpr int kWave = 64;

// Hash parameters for 32-bit keys: h = fmix32(k ^ seed) mod range.  The
// modulo uses division by an invariant integer (Granlund & Montgomery,
// "Division by Invariant Integers using Multiplication", 1994): with
// l = ceil(log2 d) and m = floor(2^(32+l) / d) + 1 (a 33-bit number, stored
// as magic = m - 2^32), q = floor(a * m / 2^(32+l)) equals floor(a / d) for
// every 32-bit a, and a mod d = a - q*d.  Two 32-bit multiplies.
struct HashParams {
    uint64_t seed;   // low 32 bits are XOR-ed into the key
    uint32_t range;  // V = d, 1 <= V < 2^32
    uint32_t magic;  // m - 2^32
    uint32_t shift;  // l - 1
    uint32_t pow2;   // V is a power of two (V = 1 included): a mod V = a & (V - 1)
};

__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b) {
    return (uint32_t)(((uint64_t)a * b) >> 32);
}

// a mod d for the divisor described by p (the branch is uniform across a launch)
__host__ __device__ __forceinline__ uint32_t mod_u32(uint32_t a, const HashParams& p) {
    if (p.pow2) return a & (p.range - 1u);
    const uint32_t t = mulhi32(a, p.magic);
    // floor((a + t) / 2^l) without overflowing 32 bits (t <= a)
    const uint32_t q = (((a - t) >> 1) + t) >> p.shift;
    return a - q * p.range;
}

__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

__host__ __device__ __forceinline__ uint64_t fmix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

// a mod d for a < 2^64 and d < 2^32 with the 128-bit M = floor((2^128-1)/d)+1
// given as (m_hi, m_lo).
__host__ __device__ __forceinline__ uint32_t fastmod_u64(uint64_t a, uint64_t m_lo, uint64_t m_hi,
                                                         uint32_t d) {
    // lowbits = (M * a) mod 2^128
    unsigned __int128 p = (unsigned __int128)m_lo * a;
    uint64_t lb_lo = (uint64_t)p;
    uint64_t lb_hi = (uint64_t)(p >> 64) + m_hi * a;
    // floor(lowbits * d / 2^128)
    unsigned __int128 t = (unsigned __int128)lb_hi * d + mulhi64(lb_lo, d);
    return (uint32_t)(t >> 64);
}

inline HashParams make_hash_params(uint64_t range, uint64_t seed) {
    HashParams p{};
    p.seed = seed;
    p.range = (uint32_t)range;
    if ((range & (range - 1)) == 0) {
        p.pow2 = 1;
        return p;
    }
    uint32_t l = 0;
    while ((1ull << l) < range) ++l;  // l = ceil(log2 d), 1 <= l <= 32
    const unsigned __int128 m = (((unsigned __int128)1) << (32 + l)) / range + 1;
    p.magic = (uint32_t)(m - (((unsigned __int128)1) << 32));
    p.shift = l - 1;
    return p;
}

// Separate parameters for 64-bit keys (the 128-bit multiplier).
struct HashParams64 {
    uint64_t seed;
    uint64_t m_lo;
    uint64_t m_hi;
    uint32_t range;
    uint32_t pow2;  // V is a power of two (V = 1 included)
};

inline HashParams64 make_hash_params64(uint64_t range, uint64_t seed) {
    HashParams64 p{};
    p.seed = seed;
    p.range = (uint32_t)range;
    unsigned __int128 all = ~(unsigned __int128)0;
    unsigned __int128 M = all / (uint32_t)range + 1;
    p.m_lo = (uint64_t)M;
    p.m_hi = (uint64_t)(M >> 64);
    p.pow2 = (range & (range - 1)) == 0;
    return p;
}

template <typename Key>
struct KeyTraits;

template <>
struct KeyTraits<uint32_t> {
    using Params = HashParams;
    static inline Params make(uint64_t range, uint64_t seed) { return make_hash_params(range, seed); }
    __host__ __device__ static __forceinline__ uint32_t bucket(uint32_t k, const Params& p) {
        return mod_u32(fmix32(k ^ (uint32_t)p.seed), p);
    }
};

template <>
struct KeyTraits<uint64_t> {
    using Params = HashParams64;
    static inline Params make(uint64_t range, uint64_t seed) { return make_hash_params64(range, seed); }
    __host__ __device__ static __forceinline__ uint32_t bucket(uint64_t k, const Params& p) {
        const uint64_t x = fmix64(k ^ p.seed);
        if (p.pow2) return (uint32_t)x & (p.range - 1u);
        return fastmod_u64(x, p.m_lo, p.m_hi, p.range);
    }
};

// Workgroups are dispatched round-robin over the 8 XCDs.  Block b of a grid
// of 8 * ceil(ub / 8) blocks takes tile (b % 8) * per + b / 8, so each XCD
// walks one contiguous range of tiles, and what neighbouring tiles read or
// write meets in that XCD's L2.  Tiles at or past ub are empty.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t ub) {
    const uint32_t per = (ub + 7) >> 3;
    return (b & 7u) * per + (b >> 3);
}

// ---------------------------------------------------------------- wave64 ---

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of `mask` at lanes below this lane
__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// inclusive scan across the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(v, d, kWave);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t o = __shfl_up(v, d, kWave);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Exclusive scan over all threads of a block (THREADS a multiple of 64).
// `tmp` must hold THREADS/64 + 1 words of LDS.  Returns the exclusive prefix
// of v; *total receives the block sum.  Contains barriers: every thread of the
// block must call it.
template <int THREADS>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
    constexpr int W = THREADS / kWave;
    const uint32_t w = threadIdx.x / kWave;
    uint32_t inc = wave_incl_scan(v);
    if (lane_id() == kWave - 1) tmp[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        uint32_t t = tmp[i];
        before += (i < (int)w) ? t : 0u;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <int THREADS>
__device__ __forceinline__ uint64_t block_excl_scan64(uint64_t v, uint64_t* tmp, uint64_t* total) {
    constexpr int W = THREADS / kWave;
    const uint32_t w = threadIdx.x / kWave;
    uint64_t inc = wave_incl_scan64(v);
    if (lane_id() == kWave - 1) tmp[w] = inc;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        uint64_t t = tmp[i];
        before += (i < (int)w) ? t : 0ull;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// Lanes of the wave whose `digit` (bits bits wide) equals this lane's, among
// the lanes in `valid`.  bits ballots; works for any digit width <= 32.
__device__ __forceinline__ uint64_t match_digit(uint32_t digit, int bits, uint64_t valid) {
    uint64_t peers = valid;
    for (int b = 0; b < bits; ++b) {
        const bool bit = (digit >> b) & 1u;
        const uint64_t bal = ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

__device__ __forceinline__ void atomic_add_relaxed(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t atomic_add_relaxed_ret(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_add_relaxed64(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace hg
