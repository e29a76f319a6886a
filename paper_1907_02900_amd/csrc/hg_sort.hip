// Stable LSD radix sort of (key, value) pairs on the device, 8-bit digits.
//
// Used where a build needs its entries grouped by a global bucket id that no
// bin fits in LDS (the heavy sets of a collection).  Per pass: each
// workgroup owns a contiguous range of whole 4096-entry tiles and counts the
// digits of its range in LDS; one workgroup scans the (digit, workgroup)
// counts digit-major, which gives every workgroup an exact base per digit;
// each workgroup then walks its tiles in order, ranks a tile stably by digit
// with wave64 ballots (rank_stable) and writes every entry at its digit's
// running base.  Equal digits keep their order, so after the last pass the
// pairs are sorted by the requested bits with ties in input order.
#include "hg_v2_device.h"

namespace hg {

namespace {

using namespace v2dev;

constexpr int kST = 256;
constexpr int kSItems = 16;
constexpr uint32_t kSTile = kST * kSItems;
constexpr uint32_t kSDigits = 256;
constexpr uint32_t kSMaxGrid = 1024;

__device__ __forceinline__ void wg_range(uint32_t n, uint32_t G, uint32_t g, uint32_t& lo,
                                         uint32_t& hi) {
    const uint32_t tiles = (n + kSTile - 1) / kSTile;
    const uint32_t per = (tiles + G - 1) / G;
    const uint64_t a = (uint64_t)g * per * kSTile, b = (uint64_t)(g + 1) * per * kSTile;
    lo = (uint32_t)(a < n ? a : n);
    hi = (uint32_t)(b < n ? b : n);
}

__global__ __launch_bounds__(kST) void k_sort_hist(const uint32_t* __restrict__ keys, uint32_t n,
                                                   uint32_t shift, uint32_t* __restrict__ hist) {
    __shared__ uint32_t cnt[kSDigits];
    const uint32_t G = gridDim.x, g = blockIdx.x;
    uint32_t lo, hi;
    wg_range(n, G, g, lo, hi);
    for (uint32_t d = threadIdx.x; d < kSDigits; d += kST) cnt[d] = 0;
    __syncthreads();
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kST) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < kSDigits; d += kST) hist[d * G + g] = cnt[d];
}

// Exclusive scan of hist[0 .. 256 * G) in place (one workgroup).
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t* __restrict__ hist, uint32_t total) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
    const uint32_t per = (total + 1023) / 1024;  // <= 256
    const uint32_t i0 = threadIdx.x * per;
    uint32_t mine = 0;
    for (uint32_t j = 0; j < per; ++j)
        if (i0 + j < total) mine += hist[i0 + j];
    uint32_t all;
    uint32_t run = block_excl_scan<1024>(mine, tmp, &all);
    for (uint32_t j = 0; j < per; ++j)
        if (i0 + j < total) {
            const uint32_t v = hist[i0 + j];
            hist[i0 + j] = run;
            run += v;
        }
}

__global__ __launch_bounds__(kST) void k_sort_scatter(const uint32_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals,
                                                      uint32_t n, uint32_t shift,
                                                      const uint32_t* __restrict__ hist,
                                                      uint32_t* __restrict__ okeys,
                                                      uint32_t* __restrict__ ovals) {
    __shared__ uint32_t base[kSDigits];
    __shared__ uint32_t wcnt[W_PART * kSDigits];
    __shared__ uint32_t dstart[kSDigits];
    __shared__ uint32_t tmp[kST / kWave + 1];
    const uint32_t G = gridDim.x, g = blockIdx.x;
    uint32_t lo, hi;
    wg_range(n, G, g, lo, hi);
    for (uint32_t d = threadIdx.x; d < kSDigits; d += kST) base[d] = hist[d * G + g];
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    for (uint32_t t0 = lo; t0 < hi; t0 += kSTile) {
        const uint32_t cnt = hi - t0 < kSTile ? hi - t0 : kSTile;
        uint32_t k[kSItems], v[kSItems], dig[kSItems], pos[kSItems];
#pragma unroll
        for (int r = 0; r < kSItems; ++r) {
            const uint32_t e = w * (kWave * kSItems) + r * kWave + lane;
            if (e < cnt) {
                k[r] = keys[t0 + e];
                v[r] = vals[t0 + e];
                dig[r] = (k[r] >> shift) & 255u;
            } else {
                k[r] = v[r] = 0;
                dig[r] = kSDigits;  // ignored by the ranking
            }
        }
        // rank_stable begins with a barrier, so base is complete before use
        rank_stable<kST, kSItems>(dig, 8, wcnt, dstart, tmp, pos);
#pragma unroll
        for (int r = 0; r < kSItems; ++r)
            if (dig[r] < kSDigits) {
                const uint32_t o = base[dig[r]] + pos[r] - dstart[dig[r]];
                okeys[o] = k[r];
                ovals[o] = v[r];
            }
        __syncthreads();
        for (uint32_t d = threadIdx.x; d < kSDigits; d += kST)
            base[d] += (d + 1 < kSDigits ? dstart[d + 1] : cnt) - dstart[d];
        __syncthreads();
    }
}

uint32_t sort_grid(uint64_t n) {
    const uint64_t tiles = (n + kSTile - 1) / kSTile;
    return (uint32_t)(tiles < kSMaxGrid ? (tiles ? tiles : 1) : kSMaxGrid);
}

}  // namespace

size_t sort_pairs_ws_bytes(uint64_t n) { return (size_t)kSDigits * sort_grid(n) * 4 + 256; }

hipError_t sort_pairs_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint64_t n,
                          uint32_t bits, void* ws, bool* in_alt, hipStream_t s) {
    *in_alt = false;
    if (n == 0 || bits == 0) return hipSuccess;
    const uint32_t G = sort_grid(n);
    uint32_t* hist = (uint32_t*)ws;
    HG_PROF("sort_pairs", s);
    bool alt = false;
    for (uint32_t shift = 0; shift < bits; shift += 8) {
        const uint32_t* ik = alt ? k1 : k0;
        const uint32_t* iv = alt ? v1 : v0;
        uint32_t* ok = alt ? k0 : k1;
        uint32_t* ov = alt ? v0 : v1;
        hipLaunchKernelGGL(k_sort_hist, dim3(G), dim3(kST), 0, s, ik, (uint32_t)n, shift, hist);
        HG_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, hist, kSDigits * G);
        HG_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_sort_scatter, dim3(G), dim3(kST), 0, s, ik, iv, (uint32_t)n, shift,
                           (const uint32_t*)hist, ok, ov);
        HG_TRY(hipGetLastError());
        alt = !alt;
    }
    *in_alt = alt;
    return hipSuccess;
}

}  // namespace hg
