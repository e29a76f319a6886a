// Device-side building blocks shared by the HashGraph kernels (gfx950, wave64).
//
//  * the hash of Eq. 1: MurmurHash3 finalisers fmix32 / fmix64 followed by an
//    exact modulo by V done with Lemire's direct-remainder method
//    (Lemire, Kaser, Kurz, "Faster Remainder by Direct Computation", 2019):
//    for a < 2^N and d < 2^L, M = ceil(2^F / d) with F >= N + L gives
//    a mod d = floor(((M * a) mod 2^F) * d / 2^F).  32-bit hashes use F = 64,
//    64-bit hashes use F = 128.
//  * wave64 helpers: lane id, masked popcount below the lane (mbcnt), ballots,
//    wave and block exclusive scans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

constexpr int kWave = 64;

// Hash parameters for 32-bit keys: h = fmix32(k ^ seed) mod range.
struct HashParams {
    uint64_t seed;   // low 32 bits are XOR-ed into the key
    uint64_t m_lo;   // Lemire multiplier floor((2^64 - 1) / range) + 1
    uint64_t m_hi;   // unused (0)
    uint32_t range;  // V, 1 <= V < 2^32
    uint32_t pad_;
};

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

// a mod d for a < 2^32 with M = floor((2^64 - 1) / d) + 1 (M wraps to 0 for
// d = 1, which correctly yields 0).
__host__ __device__ __forceinline__ uint32_t fastmod_u32(uint32_t a, uint64_t M, uint32_t d) {
    uint64_t low = M * a;
    return (uint32_t)mulhi64(low, d);
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
    p.m_lo = ~0ull / (uint32_t)range + 1ull;  // wraps to 0 for range 1
    p.m_hi = 0;
    return p;
}

// Separate parameters for 64-bit keys (the 128-bit multiplier).
struct HashParams64 {
    uint64_t seed;
    uint64_t m_lo;
    uint64_t m_hi;
    uint32_t range;
    uint32_t pad_;
};

inline HashParams64 make_hash_params64(uint64_t range, uint64_t seed) {
    HashParams64 p{};
    p.seed = seed;
    p.range = (uint32_t)range;
    unsigned __int128 all = ~(unsigned __int128)0;
    unsigned __int128 M = all / (uint32_t)range + 1;
    p.m_lo = (uint64_t)M;
    p.m_hi = (uint64_t)(M >> 64);
    return p;
}

template <typename Key>
struct KeyTraits;

template <>
struct KeyTraits<uint32_t> {
    using Params = HashParams;
    static inline Params make(uint64_t range, uint64_t seed) { return make_hash_params(range, seed); }
    __host__ __device__ static __forceinline__ uint32_t bucket(uint32_t k, const Params& p) {
        return fastmod_u32(fmix32(k ^ (uint32_t)p.seed), p.m_lo, p.range);
    }
};

template <>
struct KeyTraits<uint64_t> {
    using Params = HashParams64;
    static inline Params make(uint64_t range, uint64_t seed) { return make_hash_params64(range, seed); }
    __host__ __device__ static __forceinline__ uint32_t bucket(uint64_t k, const Params& p) {
        return fastmod_u64(fmix64(k ^ p.seed), p.m_lo, p.m_hi, p.range);
    }
};

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
