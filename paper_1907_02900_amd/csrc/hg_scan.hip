// Exclusive prefix sum (Alg. 1 PrefixSum; the CSR offset array of Sec. 3.1)
// and small fill kernels.
//
// Reduce-then-scan over tiles of 4096 counts: every tile is summed, the tile
// sums are scanned by one workgroup, and every tile is scanned again with its
// base.  Each thread owns 16 consecutive counts so the loads are 64-byte
// vectors; the per-thread totals are combined with a wave64 shuffle scan and an
// LDS pass over the waves.  Output type is uint32 (CSR offsets, wrapping) or
// uint64 (positions of join pairs, which may exceed 2^32).
#include "hg_internal.h"

namespace hg {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr uint32_t kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ void load16(const uint32_t* __restrict__ in, uint64_t base, uint64_t n,
                                       uint32_t (&v)[kScanItems]) {
    const uint32_t* p = in + base;
    if (base + kScanItems <= n && (((uintptr_t)p) & 15) == 0) {
        const uint4* q = (const uint4*)p;
#pragma unroll
        for (int j = 0; j < kScanItems / 4; ++j) {
            uint4 x = q[j];
            v[4 * j] = x.x;
            v[4 * j + 1] = x.y;
            v[4 * j + 2] = x.z;
            v[4 * j + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) v[j] = (base + j < n) ? p[j] : 0u;
    }
}

template <typename OutT>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                              uint64_t n, OutT* __restrict__ part) {
    __shared__ uint64_t tmp[kScanThreads / kWave + 1];
    uint32_t v[kScanItems];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    load16(in, base, n, v);
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) s += v[j];
    uint64_t total;
    block_excl_scan64<kScanThreads>(s, tmp, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = (OutT)total;
}

// One workgroup scans the nb tile sums in place and stores the grand total at
// part[nb].
template <typename OutT>
__global__ __launch_bounds__(1024) void k_scan_partials(OutT* __restrict__ part, uint64_t nb) {
    __shared__ uint64_t tmp[1024 / kWave + 1];
    constexpr int IT = 8;
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nb; base += 1024 * IT) {
        const uint64_t mine = base + (uint64_t)threadIdx.x * IT;
        uint64_t v[IT];
        uint64_t s = 0;
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            v[j] = (mine + j < nb) ? (uint64_t)part[mine + j] : 0ull;
            s += v[j];
        }
        uint64_t total;
        uint64_t ex = block_excl_scan64<1024>(s, tmp, &total);
        uint64_t run = carry + ex;
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            if (mine + j < nb) part[mine + j] = (OutT)run;
            run += v[j];
        }
        carry += total;
    }
    if (threadIdx.x == 0) part[nb] = (OutT)carry;
}

template <typename OutT>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* __restrict__ in,
                                                            uint64_t n,
                                                            const OutT* __restrict__ part,
                                                            OutT* __restrict__ out,
                                                            uint32_t* __restrict__ copy,
                                                            uint64_t nb) {
    __shared__ uint64_t tmp[kScanThreads / kWave + 1];
    uint32_t v[kScanItems];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    load16(in, base, n, v);
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) s += v[j];
    uint64_t total;
    uint64_t ex = block_excl_scan64<kScanThreads>(s, tmp, &total);
    uint64_t run = (uint64_t)part[blockIdx.x] + ex;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) {
            out[base + j] = (OutT)run;
            if (copy) copy[base + j] = (uint32_t)run;
        }
        run += v[j];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = part[nb];
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}

// Sum of v[0..n) added into *out (zeroed by the caller's fill): a few
// hundred workgroups, one device atomic each.
__global__ __launch_bounds__(256) void k_sum_u64(const unsigned long long* __restrict__ v,
                                                 uint64_t n, unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[256 / kWave];
    unsigned long long s = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256)
        s += v[i];
    s = wave_sum64(s);
    if (lane_id() == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long all = 0;
        for (int i = 0; i < 256 / kWave; ++i) all += red[i];
        if (all) atomicAdd(out, all);
    }
}

// Longest bucket of a CSR offset array: max over b of off[b+1] - off[b].
// One atomic max per workgroup (at most 1024 on one address).
__global__ __launch_bounds__(256) void k_max_gap(const uint32_t* __restrict__ off, uint64_t V,
                                                 uint32_t* __restrict__ out) {
    __shared__ uint32_t red[256 / kWave];
    uint32_t m = 0;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < V; b += st) {
        const uint32_t g = off[b + 1] - off[b];
        m = g > m ? g : m;
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)m, d, kWave);
        m = o > m ? o : m;
    }
    if (lane_id() == 0) red[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t all = 0;
        for (int i = 0; i < 256 / kWave; ++i) all = red[i] > all ? red[i] : all;
        if (all) atomicMax(out, all);
    }
}

template <typename OutT>
__global__ void k_set_one(OutT* p, OutT v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

}  // namespace

size_t scan_ws_bytes(uint64_t n) { return (ceil_div(n, kScanTile) + 2) * sizeof(uint64_t) + 256; }

hipError_t sum_u64(const unsigned long long* v, uint64_t n, unsigned long long* out,
                   hipStream_t s) {
    HG_TRY(fill_u32((uint32_t*)out, 2, 0u, s));
    if (n == 0) return hipSuccess;
    uint64_t blocks = ceil_div(n, 256 * 8);
    if (blocks > 256) blocks = 256;
    hipLaunchKernelGGL(k_sum_u64, dim3((uint32_t)blocks), dim3(256), 0, s, v, n, out);
    return hipGetLastError();
}

hipError_t max_bucket_len(const uint32_t* offsets, uint64_t V, uint32_t* out, hipStream_t s) {
    HG_TRY(fill_u32(out, 1, 0u, s));
    if (V == 0) return hipSuccess;
    uint64_t blocks = ceil_div(V, 256 * 8);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_max_gap, dim3((uint32_t)blocks), dim3(256), 0, s, offsets, V, out);
    return hipGetLastError();
}

hipError_t fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = ceil_div(n, 256 * 4);
    if (blocks > 8192) blocks = 8192;
    {
        HG_PROF("fill", s);
        hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p, n, v);
    }
    return hipGetLastError();
}

template <typename OutT>
hipError_t scan_excl(const uint32_t* in, uint64_t n, OutT* out, uint32_t* copy, void* ws,
                     hipStream_t s) {
    if (n == 0) {
        hipLaunchKernelGGL(k_set_one<OutT>, dim3(1), dim3(64), 0, s, out, (OutT)0);
        return hipGetLastError();
    }
    const uint64_t nb = ceil_div(n, kScanTile);
    OutT* part = (OutT*)ws;
    {
        HG_PROF("scan_reduce", s);
        hipLaunchKernelGGL(k_scan_reduce<OutT>, dim3((uint32_t)nb), dim3(kScanThreads), 0, s, in, n,
                           part);
    }
    HG_TRY(hipGetLastError());
    {
        HG_PROF("scan_partials", s);
        hipLaunchKernelGGL(k_scan_partials<OutT>, dim3(1), dim3(1024), 0, s, part, nb);
    }
    HG_TRY(hipGetLastError());
    {
        HG_PROF("scan_down", s);
        hipLaunchKernelGGL(k_scan_down<OutT>, dim3((uint32_t)nb), dim3(kScanThreads), 0, s, in, n,
                           (const OutT*)part, out, copy, nb);
    }
    return hipGetLastError();
}

template hipError_t scan_excl<uint32_t>(const uint32_t*, uint64_t, uint32_t*, uint32_t*, void*,
                                        hipStream_t);
template hipError_t scan_excl<uint64_t>(const uint32_t*, uint64_t, uint64_t*, uint32_t*, void*,
                                        hipStream_t);

}  // namespace hg
