// Deleting keys from a built table: the decremental HashGraph the paper's
// conclusion sketches, a per-bucket length array beside the offsets.
//
// After the first erase, bucket h's live entries are
// [offsets[h], offsets[h] + len[h]); the slots behind them up to offsets[h+1]
// hold stale copies of the bucket's own entries.  An erase removes every
// entry whose key is one of the given keys:
//   1. each key scans its bucket's live entries and marks the equal ones dead
//      (idempotent byte stores, so repeated keys and keys sharing a bucket
//      need no atomics) and marks the bucket touched;
//   2. each touched bucket moves its live entries down in order (the layout
//      stays stable: ids keep their order inside the bucket), sets its new
//      length and rewrites its probe index entry.  A bucket still longer
//      than kRunBucket loses its key runs (R = 0 in its entry) and is scanned by probes.
// Readers take the length into account: the index entry carries the live end,
// intersections skip stale slots of the walked table, and an export writes the
// compacted CSR of the live entries.
#include "hg_v2_device.h"

namespace hg {

namespace {

using namespace v2dev;

constexpr int kT = 256;
constexpr uint32_t kCompactBlocks = 2048;

uint32_t grid_of(uint64_t n) {
    const uint64_t g = ceil_div(n, kT);
    return (uint32_t)(g ? g : 1);
}

__global__ void k_init_len(const uint32_t* __restrict__ off, uint64_t V, uint32_t* __restrict__ len) {
    const uint64_t h = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (h < V) len[h] = off[h + 1] - off[h];
}

template <typename Key>
__global__ void k_erase_mark(const Key* __restrict__ del, uint64_t m,
                             typename KeyTraits<Key>::Params hp, const uint32_t* __restrict__ off,
                             const uint32_t* __restrict__ len, const Key* __restrict__ ekeys,
                             uint8_t* __restrict__ dead, uint8_t* __restrict__ touched) {
    const uint64_t j = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= m) return;
    const Key q = del[j];
    const uint32_t h = KeyTraits<Key>::bucket(q, hp);
    const uint32_t lo = off[h], hi = lo + len[h];
    bool any = false;
    for (uint32_t p = lo; p < hi; ++p)
        if (ekeys[p] == q) {
            dead[p] = 1;
            any = true;
        }
    if (any) touched[h] = 1;
}

// Compacts one touched bucket h; returns the number of entries it dropped.
template <typename Key>
__device__ __forceinline__ uint32_t compact_bucket(uint64_t h, const uint32_t* __restrict__ off,
                                                   uint32_t* __restrict__ len,
                                                   Key* __restrict__ ekeys,
                                                   uint32_t* __restrict__ ids,
                                                   uint8_t* __restrict__ dead,
                                                   uint4* __restrict__ head) {
    const uint32_t lo = off[h], L = len[h];
    uint32_t w = lo;
    for (uint32_t p = lo; p < lo + L; ++p) {
        if (dead[p]) {
            dead[p] = 0;
            continue;
        }
        if (w != p) {
            ekeys[w] = ekeys[p];
            ids[w] = ids[p];
        }
        ++w;
    }
    const uint32_t nl = w - lo;
    len[h] = nl;
    uint4 e = head_entry<Key>(lo, w, ekeys + lo);
    if (nl > kRunBucket) {  // no key runs any more (R = 0): probes scan the bucket
        e.z = 0;
        e.w = 0;
    }
    head[h] = e;
    return L - nl;
}

// Each thread takes groups of 16 buckets (one 16-byte load of their touched
// flags) at a stride of the grid and compacts the touched ones; `removed`
// gets the number of erased entries with one device atomic per workgroup (a
// fixed grid of at most kCompactBlocks workgroups: same-address atomics
// serialise across the chip).
template <typename Key>
__global__ __launch_bounds__(kT) void k_erase_compact(uint64_t V, const uint32_t* __restrict__ off,
                                                      uint32_t* __restrict__ len,
                                                      Key* __restrict__ ekeys,
                                                      uint32_t* __restrict__ ids,
                                                      uint8_t* __restrict__ dead,
                                                      uint8_t* __restrict__ touched,
                                                      uint4* __restrict__ head,
                                                      unsigned long long* __restrict__ removed) {
    __shared__ unsigned long long red[kT / kWave];
    unsigned long long gone = 0;
    const uint64_t groups = V / 16;
    const uint64_t stride = (uint64_t)gridDim.x * kT;
    const uint64_t t0 = (uint64_t)blockIdx.x * kT + threadIdx.x;
    for (uint64_t g = t0; g < groups; g += stride) {
        uint4 f = ((const uint4*)touched)[g];
        if ((f.x | f.y | f.z | f.w) == 0) continue;
        ((uint4*)touched)[g] = make_uint4(0u, 0u, 0u, 0u);
        const uint32_t word[4] = {f.x, f.y, f.z, f.w};
        for (int i = 0; i < 16; ++i)
            if ((word[i >> 2] >> (8 * (i & 3))) & 0xffu)
                gone += compact_bucket<Key>(g * 16 + i, off, len, ekeys, ids, dead, head);
    }
    // the last V % 16 buckets one by one
    for (uint64_t h = groups * 16 + t0; h < V; h += stride) {
        if (!touched[h]) continue;
        touched[h] = 0;
        gone += compact_bucket<Key>(h, off, len, ekeys, ids, dead, head);
    }
    gone = wave_sum64(gone);
    if (lane_id() == 0) red[threadIdx.x / kWave] = gone;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long all = 0;
        for (int i = 0; i < kT / kWave; ++i) all += red[i];
        if (all) atomicAdd(removed, all);
    }
}

// Compacted copy of the live entries: slot p holds a key of its own bucket
// (live or stale), so the key's bucket tells whether p is live.
template <typename Key>
__global__ void k_export_live(uint64_t nslots, typename KeyTraits<Key>::Params hp,
                              const uint32_t* __restrict__ off, const uint32_t* __restrict__ len,
                              const uint32_t* __restrict__ new_off, const Key* __restrict__ ekeys,
                              const uint32_t* __restrict__ ids, uint32_t* __restrict__ out_ids,
                              Key* __restrict__ out_keys) {
    const uint64_t p = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= nslots) return;
    const Key k = ekeys[p];
    const uint32_t h = KeyTraits<Key>::bucket(k, hp);
    const uint32_t r = (uint32_t)p - off[h];
    if (r >= len[h]) return;
    const uint32_t o = new_off[h] + r;
    if (out_ids) out_ids[o] = ids[p];
    if (out_keys) out_keys[o] = k;
}

}  // namespace

hipError_t init_lengths(const uint32_t* offsets, uint64_t V, uint32_t* len, hipStream_t s) {
    hipLaunchKernelGGL(k_init_len, dim3(grid_of(V)), dim3(kT), 0, s, offsets, V, len);
    return hipGetLastError();
}

template <typename Key>
hipError_t run_erase(const TableDev& t, uint32_t* len, uint8_t* dead, uint8_t* touched,
                     uint4* head, const Key* del, uint64_t m, unsigned long long* d_removed,
                     hipStream_t s) {
    auto hp = KeyTraits<Key>::make(t.V, t.seed);
    if (m) {
        HG_PROF("erase_mark", s);
        hipLaunchKernelGGL(k_erase_mark<Key>, dim3(grid_of(m)), dim3(kT), 0, s, del, m, hp,
                           t.offsets, (const uint32_t*)len, (const Key*)t.keys, dead, touched);
        HG_TRY(hipGetLastError());
    }
    HG_PROF("erase_compact", s);
    const uint32_t g16 = grid_of(ceil_div(t.V, 16));
    const uint32_t cb = g16 < kCompactBlocks ? g16 : kCompactBlocks;
    hipLaunchKernelGGL(k_erase_compact<Key>, dim3(cb), dim3(kT), 0, s, t.V, t.offsets,
                       len, (Key*)t.keys, (uint32_t*)t.ids, dead, touched, head, d_removed);
    return hipGetLastError();
}

template <typename Key>
hipError_t run_export_live(const TableDev& t, const uint32_t* len, const uint32_t* new_off,
                           uint32_t* out_ids, Key* out_keys, hipStream_t s) {
    if (t.n == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(t.V, t.seed);
    hipLaunchKernelGGL(k_export_live<Key>, dim3(grid_of(t.n)), dim3(kT), 0, s, t.n, hp,
                       t.offsets, len, new_off, (const Key*)t.keys, t.ids, out_ids, out_keys);
    return hipGetLastError();
}

#define HG_ERASE_INST(Key)                                                                      \
    template hipError_t run_erase<Key>(const TableDev&, uint32_t*, uint8_t*, uint8_t*, uint4*, \
                                       const Key*, uint64_t, unsigned long long*, hipStream_t); \
    template hipError_t run_export_live<Key>(const TableDev&, const uint32_t*, const uint32_t*, \
                                             uint32_t*, Key*, hipStream_t);
HG_ERASE_INST(uint32_t)
HG_ERASE_INST(uint64_t)
#undef HG_ERASE_INST

}  // namespace hg
