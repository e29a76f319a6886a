// Scatter by a permutation: out[ids[p]] = vals[p] for every p < n, where ids
// holds each index of [0, n) exactly once (a table's edge ids).  Used to turn
// Alg. 3's counts, which come out in B's edge order, into counts by B's input
// index.
//
// A direct scatter writes one random 4-byte word per entry, and random
// partial-line writes beyond the L2 run at a small fraction of the HBM rate.
// Here the (id, value) pairs are first partitioned by the top bits of the id
// into W <= 256 windows of 2^wshift consecutive ids -- per-tile LDS
// histograms written digit-major, one workgroup per window scanning its
// column, and a tile partition ranked with LDS atomics -- so that window d's
// pairs sit in [d << wshift, (d+1) << wshift) of a staging array (each id
// occurs once, so a window never holds more than 2^wshift pairs).  Each
// window, whose 4 << wshift bytes of output fit in one XCD's 4 MiB L2, is then
// written by workgroups of a single XCD: the writes stay random, but they
// merge into whole lines in that L2.
#include "hg_internal.h"

namespace hg {

namespace {

constexpr int kScThreads = 256;
constexpr int kScItems = 16;
constexpr uint32_t kScTile = kScThreads * kScItems;
constexpr uint32_t kScMaxWindowBits = 8;   // at most 256 windows
constexpr uint32_t kScDirectMax = 1u << 20;  // below this a direct scatter stays in L2

struct ScPlan {
    uint32_t wshift = 0;  // ids per window = 2^wshift
    uint32_t W = 0;       // windows
    uint32_t T = 0;       // tiles of kScTile entries
    uint64_t staged = 0;  // staging entries (W << wshift)
};

ScPlan sc_plan(uint64_t n) {
    ScPlan p;
    const uint32_t b = log2_ceil(n ? n : 1);
    const uint32_t wb = b < kScMaxWindowBits ? b : kScMaxWindowBits;
    p.wshift = b - wb;
    p.W = (uint32_t)ceil_div(n ? n : 1, 1ull << p.wshift);
    p.T = (uint32_t)ceil_div(n, kScTile);
    p.staged = (uint64_t)p.W << p.wshift;
    return p;
}

// Tile t's count of each window, stored digit-major: mat[d * T + t].
__global__ __launch_bounds__(kScThreads) void k_sc_hist(const uint32_t* __restrict__ ids,
                                                        uint64_t n, uint32_t wshift, uint32_t W,
                                                        uint32_t T, uint32_t* __restrict__ mat) {
    __shared__ uint32_t cnt[1u << kScMaxWindowBits];
    const uint32_t t = blockIdx.x;
    for (uint32_t d = threadIdx.x; d < W; d += kScThreads) cnt[d] = 0;
    __syncthreads();
    const uint64_t begin = (uint64_t)t * kScTile;
#pragma unroll
    for (int r = 0; r < kScItems; ++r) {
        const uint64_t p = begin + (uint64_t)r * kScThreads + threadIdx.x;
        if (p < n) {
            const uint32_t d = ids[p] >> wshift;
            if (d < W) atomicAdd(&cnt[d], 1u);
        }
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < W; d += kScThreads) mat[(size_t)d * T + t] = cnt[d];
}

// One workgroup per window d: mat[d * T + t] becomes the staging position of
// tile t's first pair of window d, (d << wshift) + the pairs of window d in
// tiles before t.
__global__ __launch_bounds__(1024) void k_sc_scan(uint32_t* __restrict__ mat, uint32_t T,
                                                  uint32_t wshift) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
    const uint32_t d = blockIdx.x;
    uint32_t* col = mat + (size_t)d * T;
    uint32_t carry = d << wshift;
    for (uint32_t t0 = 0; t0 < T; t0 += 1024 * 4) {
        uint32_t v[4], s = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t t = t0 + threadIdx.x * 4 + j;
            v[j] = t < T ? col[t] : 0u;
            s += v[j];
        }
        uint32_t all;
        uint32_t run = carry + block_excl_scan<1024>(s, tmp, &all);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t t = t0 + threadIdx.x * 4 + j;
            if (t < T) col[t] = run;
            run += v[j];
        }
        carry += all;
    }
}

// Tile t's pairs grouped by window (order inside a window unspecified) and
// written to their staging positions.
__global__ __launch_bounds__(kScThreads) void k_sc_part(const uint32_t* __restrict__ ids,
                                                        const uint32_t* __restrict__ vals,
                                                        uint64_t n, uint32_t wshift, uint32_t W,
                                                        uint32_t T, const uint32_t* __restrict__ mat,
                                                        uint32_t* __restrict__ st_ids,
                                                        uint32_t* __restrict__ st_vals) {
    __shared__ uint32_t cnt[1u << kScMaxWindowBits];
    __shared__ uint32_t dstart[1u << kScMaxWindowBits];
    __shared__ uint32_t gbase[1u << kScMaxWindowBits];
    __shared__ uint32_t tmp[kScThreads / kWave + 1];
    __shared__ uint32_t sid[kScTile];
    __shared__ uint32_t sval[kScTile];
    __shared__ uint8_t sdig[kScTile];
    const uint32_t t = blockIdx.x;
    const uint64_t begin = (uint64_t)t * kScTile;
    const uint32_t cntp = (uint32_t)(n - begin < kScTile ? n - begin : kScTile);
    for (uint32_t d = threadIdx.x; d < W; d += kScThreads) cnt[d] = 0;
    __syncthreads();
    uint32_t id[kScItems], v[kScItems], dig[kScItems], pos[kScItems];
#pragma unroll
    for (int r = 0; r < kScItems; ++r) {
        const uint32_t e = (uint32_t)r * kScThreads + threadIdx.x;
        if (e < cntp) {
            id[r] = ids[begin + e];
            v[r] = vals[begin + e];
            dig[r] = id[r] >> wshift;
        } else {
            id[r] = v[r] = 0;
            dig[r] = W;
        }
        if (dig[r] < W) pos[r] = atomicAdd(&cnt[dig[r]], 1u);
    }
    __syncthreads();
    // exclusive scan of the tile's window counts (W <= 256 = kScThreads)
    const uint32_t c = threadIdx.x < W ? cnt[threadIdx.x] : 0u;
    uint32_t all;
    const uint32_t ex = block_excl_scan<kScThreads>(c, tmp, &all);
    if (threadIdx.x < W) {
        dstart[threadIdx.x] = ex;
        gbase[threadIdx.x] = mat[(size_t)threadIdx.x * T + t];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kScItems; ++r) {
        if (dig[r] < W) {
            const uint32_t q = dstart[dig[r]] + pos[r];
            sid[q] = id[r];
            sval[q] = v[r];
            sdig[q] = (uint8_t)dig[r];
        }
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < all; q += kScThreads) {
        const uint32_t d = sdig[q];
        const uint64_t o = (uint64_t)gbase[d] + (q - dstart[d]);
        if ((o >> wshift) == d) {  // inside window d (always, for a permutation)
            st_ids[o] = sid[q];
            st_vals[o] = sval[q];
        }
    }
}

// Window d, chunk c (kScTile staged pairs): out[id] = value.  Workgroup b
// runs on XCD b % 8 (round-robin dispatch); the workgroups of one XCD walk
// its windows x, x + 8, x + 16, ... in order, so the writes of a window land
// in one L2 while it is being written.
__global__ __launch_bounds__(kScThreads) void k_sc_apply(const uint32_t* __restrict__ st_ids,
                                                         const uint32_t* __restrict__ st_vals,
                                                         uint64_t n, uint32_t wshift, uint32_t W,
                                                         uint32_t chunks,
                                                         uint32_t* __restrict__ out) {
    const uint32_t x = blockIdx.x & 7u, s = blockIdx.x >> 3;
    const uint32_t d = x + 8u * (s / chunks), c = s % chunks;
    if (d >= W) return;
    const uint64_t w0 = (uint64_t)d << wshift;
    const uint64_t wn = n - w0 < (1ull << wshift) ? n - w0 : (1ull << wshift);
    const uint64_t begin = (uint64_t)c * kScTile;
#pragma unroll
    for (int r = 0; r < kScItems; ++r) {
        const uint64_t e = begin + (uint64_t)r * kScThreads + threadIdx.x;
        if (e < wn) {
            const uint32_t id = st_ids[w0 + e];
            if (id < n) out[id] = st_vals[w0 + e];
        }
    }
}

__global__ void k_sc_direct(const uint32_t* __restrict__ ids, const uint32_t* __restrict__ vals,
                            uint64_t n, uint32_t* __restrict__ out) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (; p < n; p += st) {
        const uint32_t id = ids[p];
        if (id < n) out[id] = vals[p];
    }
}

size_t sc_layout(void* ws, const ScPlan& p, uint32_t** mat, uint32_t** st_ids,
                 uint32_t** st_vals) {
    Carver c(ws);
    *mat = c.take<uint32_t>((size_t)p.W * p.T);
    *st_ids = c.take<uint32_t>(p.staged);
    *st_vals = c.take<uint32_t>(p.staged);
    return c.off + 256;
}

}  // namespace

size_t scatter_perm_ws_bytes(uint64_t n) {
    if (n <= kScDirectMax) return 256;
    uint32_t *a, *b, *c;
    return sc_layout(nullptr, sc_plan(n), &a, &b, &c);
}

hipError_t scatter_perm(const uint32_t* ids, const uint32_t* vals, uint64_t n, uint32_t* out,
                        void* ws, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (n <= kScDirectMax) {
        HG_PROF("scatter_direct", s);
        const uint64_t g = ceil_div(n, 256 * 4);
        hipLaunchKernelGGL(k_sc_direct, dim3((uint32_t)(g > 4096 ? 4096 : g)), dim3(256), 0, s,
                           ids, vals, n, out);
        return hipGetLastError();
    }
    const ScPlan p = sc_plan(n);
    uint32_t *mat, *st_ids, *st_vals;
    sc_layout(ws, p, &mat, &st_ids, &st_vals);
    {
        HG_PROF("scatter_hist", s);
        hipLaunchKernelGGL(k_sc_hist, dim3(p.T), dim3(kScThreads), 0, s, ids, n, p.wshift, p.W,
                           p.T, mat);
    }
    HG_TRY(hipGetLastError());
    {
        HG_PROF("scatter_scan", s);
        hipLaunchKernelGGL(k_sc_scan, dim3(p.W), dim3(1024), 0, s, mat, p.T, p.wshift);
    }
    HG_TRY(hipGetLastError());
    {
        HG_PROF("scatter_part", s);
        hipLaunchKernelGGL(k_sc_part, dim3(p.T), dim3(kScThreads), 0, s, ids, vals, n, p.wshift,
                           p.W, p.T, (const uint32_t*)mat, st_ids, st_vals);
    }
    HG_TRY(hipGetLastError());
    const uint32_t chunks = (uint32_t)ceil_div(1ull << p.wshift, kScTile);
    const uint64_t grid = 8ull * ceil_div(p.W, 8) * chunks;
    {
        HG_PROF("scatter_apply", s);
        hipLaunchKernelGGL(k_sc_apply, dim3((uint32_t)grid), dim3(kScThreads), 0, s,
                           (const uint32_t*)st_ids, (const uint32_t*)st_vals, n, p.wshift, p.W,
                           chunks, out);
    }
    return hipGetLastError();
}

}  // namespace hg
