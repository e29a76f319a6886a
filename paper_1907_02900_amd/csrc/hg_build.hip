// HashGraph builds on gfx950: Eq. 1 hashing, Alg. 1 (V1) and Alg. 2 (V2).
//
// V1 (Alg. 1) is written as the paper states it: a global atomic histogram,
// a prefix sum, and an atomic scatter that takes each key's slot from a cursor
// array initialised to the offsets.  On MI355X every device-scope atomic is
// executed beyond the L2, so V1 is bound by atomic throughput.
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

template <typename Key>
hipError_t run_histogram(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* counts,
                         uint32_t block, hipStream_t s) {
    if (!block) block = 256;
    HG_TRY(fill_u32(counts, V, 0u, s));
    if (n == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(V, seed);
    {
        HG_PROF("v1_hist_global", s);
        hipLaunchKernelGGL(k_hist_global<Key>, dim3(stream_grid(n, block)), dim3(block), 0, s, keys, n,
                           hp, counts);
    }
    return hipGetLastError();
}

template <typename Key>
hipError_t run_build_v1(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* offsets,
                        uint32_t* ids, Key* ekeys, void* ws, uint32_t block, hipStream_t s) {
    if (!block) block = 256;
    Carver c(ws);
    uint32_t* counts = c.take<uint32_t>(V);
    void* scan_ws = c.take<char>(scan_ws_bytes(V));
    HG_TRY(run_histogram<Key>(keys, n, V, seed, counts, block, s));
    // offsets = exclusive scan; the counts become the cursors (Alg. 1, fifth
    // loop re-zeroes them; here they start at the offsets so the scatter's
    // atomic returns the absolute slot).
    HG_TRY(scan_excl<uint32_t>(counts, V, offsets, counts, scan_ws, s));
    if (n == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(V, seed);
    {
        HG_PROF("v1_scatter", s);
        hipLaunchKernelGGL(k_scatter_v1<Key>, dim3(stream_grid(n, block)), dim3(block), 0, s, keys, n,
                           hp, counts, ids, ekeys);
    }
    return hipGetLastError();
}

#define HG_INST(Key)                                                                              \
    template hipError_t run_hash<Key>(const Key*, uint64_t, uint64_t, uint64_t, uint32_t*,       \
                                      hipStream_t);                                              \
    template hipError_t run_histogram<Key>(const Key*, uint64_t, uint64_t, uint64_t, uint32_t*,  \
                                           uint32_t, hipStream_t);                               \
    template hipError_t run_build_v1<Key>(const Key*, uint64_t, uint64_t, uint64_t, uint32_t*,   \
                                          uint32_t*, Key*, void*, uint32_t, hipStream_t);
HG_INST(uint32_t)
HG_INST(uint64_t)

}  // namespace hg
