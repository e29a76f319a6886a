// HashGraph builds on gfx950: Eq. 1 hashing, Alg. 1 (V1) and Alg. 2 (V2).
//
// V1 (Alg. 1): a global atomic histogram, a prefix sum, and an atomic scatter
// that takes each key's slot from a cursor array initialised to the offsets.
// On MI355X every device-scope atomic is executed beyond the L2, so V1 is
// bound by atomic throughput; by default the atomics of lanes that share a
// bucket are merged inside each wave (the paper's one-atomic-per-key loops
// remain selectable).
//
// V2 (Alg. 2) lives in hg_v2.hip.
#include "hg_internal.h"

namespace hg {

// ============================================================== hashing ===

template <typename Key>
__global__ void k_hash(const Key* __restrict__ keys, uint64_t n,
                       typename KeyTraits<Key>::Params hp, uint32_t* __restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) out[i] = KeyTraits<Key>::bucket(keys[i], hp);
}

static uint32_t stream_grid(uint64_t n, uint32_t block) {
    uint64_t g = ceil_div(n, (uint64_t)block * 4);
    if (g > 4096) g = 4096;
    if (g == 0) g = 1;
    return (uint32_t)g;
}

template <typename Key>
hipError_t run_hash(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* out,
                    hipStream_t s) {
    if (n == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(V, seed);
    {
        HG_PROF("hash", s);
        hipLaunchKernelGGL(k_hash<Key>, dim3(stream_grid(n, 256)), dim3(256), 0, s, keys, n, hp, out);
    }
    return hipGetLastError();
}

// ================================================================== V1 ===

// The paper's loops as printed: one device-scope atomic per key.
template <typename Key>
__global__ void k_hist_global(const Key* __restrict__ keys, uint64_t n,
                              typename KeyTraits<Key>::Params hp, uint32_t* __restrict__ counts) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) atomic_add_relaxed(&counts[KeyTraits<Key>::bucket(keys[i], hp)], 1u);
}

template <typename Key>
__global__ void k_scatter_v1(const Key* __restrict__ keys, uint64_t n,
                             typename KeyTraits<Key>::Params hp, uint32_t* __restrict__ cursor,
                             uint32_t* __restrict__ ids, Key* __restrict__ ekeys) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        const Key k = keys[i];
        const uint32_t pos = atomic_add_relaxed_ret(&cursor[KeyTraits<Key>::bucket(k, hp)], 1u);
        if (pos < n) {  // always true when the counts are exact
            ekeys[pos] = k;
            ids[pos] = (uint32_t)i;
        }
    }
}

// Wave-aggregated forms (the default).  A wave takes 64 consecutive keys at
// a time; the lanes whose keys fall into the same bucket find each other with
// one ballot per bit of the bucket index (bits = ceil(log2 V)), and the lowest
// of them issues a single atomic that adds the group's size.  In the scatter
// that lane hands the returned cursor to the group, whose lanes take
// consecutive slots after it.  Uniform keys rarely share a bucket inside a
// wave and pay only the ballots; skewed keys (a hot key held by many lanes)
// turn many atomics on one address into one.
template <typename Key>
__global__ void k_hist_wave(const Key* __restrict__ keys, uint64_t n,
                            typename KeyTraits<Key>::Params hp, int bits,
                            uint32_t* __restrict__ counts) {
    const uint32_t lane = lane_id();
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; w0 < n; w0 += st) {
        const uint64_t i = w0 + lane;
        const bool valid = i < n;
        const uint32_t h = valid ? KeyTraits<Key>::bucket(keys[i], hp) : 0u;
        const uint64_t peers = match_digit(h, bits, ballot(valid));
        if (valid && mbcnt(peers) == 0) atomic_add_relaxed(&counts[h], (uint32_t)__popcll(peers));
    }
}

template <typename Key>
__global__ void k_scatter_wave(const Key* __restrict__ keys, uint64_t n,
                               typename KeyTraits<Key>::Params hp, int bits,
                               uint32_t* __restrict__ cursor, uint32_t* __restrict__ ids,
                               Key* __restrict__ ekeys) {
    const uint32_t lane = lane_id();
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; w0 < n; w0 += st) {
        const uint64_t i = w0 + lane;
        const bool valid = i < n;
        const Key k = valid ? keys[i] : Key(0);
        const uint32_t h = valid ? KeyTraits<Key>::bucket(k, hp) : 0u;
        const uint64_t peers = match_digit(h, bits, ballot(valid));
        const uint32_t rank = mbcnt(peers);
        uint32_t base = 0;
        if (valid && rank == 0) base = atomic_add_relaxed_ret(&cursor[h], (uint32_t)__popcll(peers));
        // every lane reads its group leader's cursor (invalid lanes their own)
        const int leader = valid ? (int)__builtin_ctzll(peers) : (int)lane;
        base = (uint32_t)__shfl((int)base, leader, kWave);
        const uint32_t pos = base + rank;
        if (valid && pos < n) {  // always true when the counts are exact
            ekeys[pos] = k;
            ids[pos] = (uint32_t)i;
        }
    }
}

template <typename Key>
hipError_t run_histogram(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* counts,
                         uint32_t block, bool plain, hipStream_t s) {
    if (!block) block = 256;
    HG_TRY(fill_u32(counts, V, 0u, s));
    if (n == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(V, seed);
    if (plain) {
        HG_PROF("v1_hist_global", s);
        hipLaunchKernelGGL(k_hist_global<Key>, dim3(stream_grid(n, block)), dim3(block), 0, s, keys, n,
                           hp, counts);
    } else {
        HG_PROF("v1_hist_wave", s);
        hipLaunchKernelGGL(k_hist_wave<Key>, dim3(stream_grid(n, block)), dim3(block), 0, s, keys, n,
                           hp, (int)log2_ceil(V), counts);
    }
    return hipGetLastError();
}

template <typename Key>
hipError_t run_build_v1(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* offsets,
                        uint32_t* ids, Key* ekeys, void* ws, uint32_t block, bool plain,
                        hipStream_t s) {
    if (!block) block = 256;
    Carver c(ws);
    uint32_t* counts = c.take<uint32_t>(V);
    void* scan_ws = c.take<char>(scan_ws_bytes(V));
    HG_TRY(run_histogram<Key>(keys, n, V, seed, counts, block, plain, s));
    // offsets = exclusive scan; the counts become the cursors (Alg. 1, fifth
    // loop re-zeroes them; here they start at the offsets so the scatter's
    // atomic returns the absolute slot).
    HG_TRY(scan_excl<uint32_t>(counts, V, offsets, counts, scan_ws, s));
    if (n == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(V, seed);
    if (plain) {
        HG_PROF("v1_scatter", s);
        hipLaunchKernelGGL(k_scatter_v1<Key>, dim3(stream_grid(n, block)), dim3(block), 0, s, keys, n,
                           hp, counts, ids, ekeys);
    } else {
        HG_PROF("v1_scatter_wave", s);
        hipLaunchKernelGGL(k_scatter_wave<Key>, dim3(stream_grid(n, block)), dim3(block), 0, s, keys,
                           n, hp, (int)log2_ceil(V), counts, ids, ekeys);
    }
    return hipGetLastError();
}

#define HG_INST(Key)                                                                              \
    template hipError_t run_hash<Key>(const Key*, uint64_t, uint64_t, uint64_t, uint32_t*,       \
                                      hipStream_t);                                              \
    template hipError_t run_histogram<Key>(const Key*, uint64_t, uint64_t, uint64_t, uint32_t*,  \
                                           uint32_t, bool, hipStream_t);                         \
    template hipError_t run_build_v1<Key>(const Key*, uint64_t, uint64_t, uint64_t, uint32_t*,   \
                                          uint32_t*, Key*, void*, uint32_t, bool, hipStream_t);
HG_INST(uint32_t)
HG_INST(uint64_t)

}  // namespace hg
