// Random-transaction micro-roofline.  The probe of Sec. 3.4 makes one random
// 16-byte read per query (its bucket's index entry) and V1 (Alg. 1) one random
// atomic add per key, so their ceilings are not the streaming bandwidth but
// the rate of independent random transactions the memory system sustains.
// These kernels measure that rate over a power-of-two footprint: every thread
// issues kItems independent accesses at addresses drawn by a hash of the
// access number, and only then combines the loaded values, so the loads
// overlap as they do in the probe.
#include "hashgraph.h"
#include "hg_internal.h"

namespace hg {

namespace {

constexpr int kT = 256;
constexpr int kItems = 8;

__device__ __forceinline__ uint64_t slot_of(uint64_t i, uint32_t seed, uint64_t mask) {
    const uint64_t x = fmix64(i * 0x9E3779B97F4A7C15ull + seed);
    return x & mask;
}

__global__ __launch_bounds__(kT) void k_rand_read4(const uint32_t* __restrict__ buf, uint64_t mask,
                                                   uint64_t n, uint32_t seed,
                                                   uint32_t* __restrict__ sink) {
    const uint64_t base = (uint64_t)blockIdx.x * kT * kItems + threadIdx.x;
    uint32_t v[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint64_t i = base + (uint64_t)r * kT;
        v[r] = i < n ? buf[slot_of(i, seed, mask)] : 0u;
    }
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) acc ^= v[r];
    if (acc == 0x9E3779B9u) sink[0] = acc;  // keeps the loads; the buffer holds zeros
}

__global__ __launch_bounds__(kT) void k_rand_read16(const uint4* __restrict__ buf, uint64_t mask,
                                                    uint64_t n, uint32_t seed,
                                                    uint32_t* __restrict__ sink) {
    const uint64_t base = (uint64_t)blockIdx.x * kT * kItems + threadIdx.x;
    uint4 v[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint64_t i = base + (uint64_t)r * kT;
        v[r] = i < n ? buf[slot_of(i, seed, mask)] : make_uint4(0u, 0u, 0u, 0u);
    }
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) acc ^= v[r].x ^ v[r].y ^ v[r].z ^ v[r].w;
    if (acc == 0x9E3779B9u) sink[0] = acc;
}

__global__ __launch_bounds__(kT) void k_rand_atomic4(uint32_t* __restrict__ buf, uint64_t mask,
                                                     uint64_t n, uint32_t seed) {
    const uint64_t base = (uint64_t)blockIdx.x * kT * kItems + threadIdx.x;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint64_t i = base + (uint64_t)r * kT;
        if (i < n) atomicAdd(&buf[slot_of(i, seed, mask)], 1u);
    }
}

hipError_t launch(int kind, void* buf, uint64_t words, uint64_t n, uint32_t seed, uint32_t* sink,
                  hipStream_t s) {
    const uint64_t g = ceil_div(n, (uint64_t)kT * kItems);
    const dim3 grid((uint32_t)g), block(kT);
    if (kind == HG_MICRO_READ4)
        hipLaunchKernelGGL(k_rand_read4, grid, block, 0, s, (const uint32_t*)buf, words - 1, n,
                           seed, sink);
    else if (kind == HG_MICRO_READ16)
        hipLaunchKernelGGL(k_rand_read16, grid, block, 0, s, (const uint4*)buf, words / 4 - 1, n,
                           seed, sink);
    else
        hipLaunchKernelGGL(k_rand_atomic4, grid, block, 0, s, (uint32_t*)buf, words - 1, n, seed);
    return hipGetLastError();
}

}  // namespace

}  // namespace hg

using namespace hg;

hg_status hg_random_access_rate(int kind, uint64_t footprint_bytes, uint64_t accesses,
                                double* h_ms, hipStream_t stream) {
    if (!h_ms || (kind != HG_MICRO_READ4 && kind != HG_MICRO_READ16 && kind != HG_MICRO_ATOMIC4))
        return HG_ERR_INVALID_ARG;
    if (footprint_bytes < 4096 || (footprint_bytes & (footprint_bytes - 1)) ||
        accesses == 0 || accesses > (1ull << 40))
        return HG_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return HG_ERR_DEVICE;
    void* buf = nullptr;
    uint32_t* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hg_status st = HG_OK;
    float ms = 0.f;
    const uint64_t words = footprint_bytes / 4;
    if (hipMalloc(&buf, footprint_bytes) != hipSuccess) return HG_ERR_OOM;
    if (hipMalloc((void**)&sink, 256) != hipSuccess) {
        (void)hipFree(buf);
        return HG_ERR_OOM;
    }
    if (hipMemsetAsync(buf, 0, footprint_bytes, stream) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        launch(kind, buf, words, accesses, 1u, sink, stream) != hipSuccess ||  // warm-up
        hipEventRecord(e0, stream) != hipSuccess ||
        launch(kind, buf, words, accesses, 2u, sink, stream) != hipSuccess ||
        hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        st = HG_ERR_DEVICE;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(stream);
    (void)hipFree(sink);
    (void)hipFree(buf);
    if (st == HG_OK) *h_ms = ms;
    return st;
}
