// Key-run summaries of long buckets: exact probing under skew.
//
// Probe-Standard (Sec. 3.4) scans a query's whole bucket.  When many entries
// share a bucket -- heavy duplication, or Zipf keys where one key holds a
// large share of the input -- every probe of that bucket pays its full
// length, so a skewed join costs as much as the number of matching pairs.
// For each bucket longer than kRunBucket the table therefore also keeps the
// bucket's distinct keys in ascending order, each with the number of entries
// holding it and the start of its run in `kperm`, a copy of the bucket's ids
// grouped by key (ids ascending inside each group, as in the bucket).  The
// bucket's probe index entry points at its runs.  A probe of a long bucket
// binary-searches the runs; its pairs are the ids of one run.  Counts and
// pairs are exactly those of a scan.
//
// Construction: every final bin of the build tallied its long buckets; a scan
// of the tallies sizes the summary, a per-bin pass lists the long buckets,
// and their entries are gathered with the sort key (list index, key), sorted
// (a device radix sort, stable, so equal keys keep ascending ids), and a
// flag/scan pass marks the runs.
#include <rocprim/device/device_radix_sort.hpp>

#include "hg_internal.h"

namespace hg {

namespace {

constexpr int kThreads = 256;

uint32_t blocks_for(uint64_t n) {
    const uint64_t g = ceil_div(n, kThreads);
    return (uint32_t)(g ? g : 1);
}

uint32_t bits_for(uint64_t count) {  // bits to hold values 0 .. count-1
    uint32_t b = 0;
    while (b < 32 && (1ull << b) < count) ++b;
    return b;
}

__global__ void k_long_len(const uint32_t* __restrict__ off, const uint32_t* __restrict__ list,
                           uint32_t nlong, uint32_t* __restrict__ len) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i < nlong) {
        const uint32_t b = list[i];
        len[i] = off[b + 1] - off[b];
    }
}

// largest i < nlong with base[i] <= j
__device__ __forceinline__ uint32_t owner(const uint32_t* __restrict__ base, uint32_t nlong,
                                          uint32_t j) {
    uint32_t lo = 0, hi = nlong;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Entry j of the gathered long buckets: its list index, edge position and key.
// 32-bit keys: one 64-bit sort key (list index << 32 | key).
__global__ void k_gather32(const uint32_t* __restrict__ off, const uint32_t* __restrict__ list,
                           const uint32_t* __restrict__ base, uint32_t nlong, uint32_t total,
                           const uint32_t* __restrict__ ekeys, uint64_t* __restrict__ sk,
                           uint32_t* __restrict__ pos) {
    const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= total) return;
    const uint32_t i = owner(base, nlong, j);
    const uint32_t p = off[list[i]] + (j - base[i]);
    sk[j] = ((uint64_t)i << 32) | ekeys[p];
    pos[j] = p;
}

// 64-bit keys: the key and the list index are sorted in two stable passes.
__global__ void k_gather64(const uint32_t* __restrict__ off, const uint32_t* __restrict__ list,
                           const uint32_t* __restrict__ base, uint32_t nlong, uint32_t total,
                           const uint64_t* __restrict__ ekeys, uint64_t* __restrict__ sk,
                           uint32_t* __restrict__ idx, uint32_t* __restrict__ seg,
                           uint32_t* __restrict__ pos) {
    const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= total) return;
    const uint32_t i = owner(base, nlong, j);
    const uint32_t p = off[list[i]] + (j - base[i]);
    sk[j] = ekeys[p];
    idx[j] = j;
    seg[j] = i;
    pos[j] = p;
}

// after the key sort: list index of each key-sorted entry, and its position
__global__ void k_seg_of(const uint32_t* __restrict__ idx, const uint32_t* __restrict__ seg,
                         uint32_t total, uint32_t* __restrict__ seg2, uint32_t* __restrict__ ord) {
    const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= total) return;
    seg2[j] = seg[idx[j]];
    ord[j] = j;
}

// Sorted view: entry j has list index sseg[j], key skey[j], edge position spos[j].
template <typename Key>
struct Sorted {
    const uint32_t* sseg;  // 32-bit keys: null, taken from the composite
    const Key* skey;
    const uint64_t* comp;  // 32-bit keys: (list index << 32 | key)
    const uint32_t* spos;
    const uint32_t* ord;   // 64-bit keys: j -> key-sorted index (null for 32-bit keys)
};

template <typename Key>
__device__ __forceinline__ void sorted_at(const Sorted<Key>& s, uint32_t j, uint32_t& seg, Key& k,
                                          uint32_t& p) {
    if constexpr (sizeof(Key) == 4) {
        const uint64_t c = s.comp[j];
        seg = (uint32_t)(c >> 32);
        k = (Key)(uint32_t)c;
        p = s.spos[j];
    } else {
        const uint32_t t = s.ord[j];
        seg = s.sseg[j];
        k = s.skey[t];
        p = s.spos[t];
    }
}

template <typename Key>
__global__ void k_run_flags(Sorted<Key> s, uint32_t total, uint32_t* __restrict__ flag) {
    const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= total) return;
    uint32_t seg, p;
    Key k;
    sorted_at(s, j, seg, k, p);
    uint32_t f = 1;
    if (j) {
        uint32_t seg0, p0;
        Key k0;
        sorted_at(s, j - 1, seg0, k0, p0);
        f = (seg0 != seg || k0 != k) ? 1u : 0u;
    }
    flag[j] = f;
}

template <typename Key>
__global__ void k_run_emit(Sorted<Key> s, uint32_t total, const uint32_t* __restrict__ flag,
                           const uint32_t* __restrict__ rid, const uint32_t* __restrict__ off,
                           const uint32_t* __restrict__ list, const uint32_t* __restrict__ base,
                           const uint32_t* __restrict__ ids, Key* __restrict__ run_key,
                           uint32_t* __restrict__ run_pos, uint32_t* __restrict__ rstart,
                           uint32_t* __restrict__ first_run, uint32_t* __restrict__ kperm) {
    const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= total) return;
    uint32_t seg, p;
    Key k;
    sorted_at(s, j, seg, k, p);
    const uint32_t at = off[list[seg]] + (j - base[seg]);  // key-grouped slot in the bucket
    kperm[at] = ids[p];
    if (flag[j]) {
        const uint32_t r = rid[j];
        run_key[r] = k;
        run_pos[r] = at;
        rstart[r] = j;
        if (j == base[seg]) first_run[seg] = r;
    }
}

__global__ void k_run_cnt(const uint32_t* __restrict__ rstart, const uint32_t* __restrict__ nruns,
                          uint32_t total, uint32_t* __restrict__ run_cnt) {
    const uint32_t r = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t R = *nruns;
    if (r >= R) return;
    run_cnt[r] = ((r + 1 < R) ? rstart[r + 1] : total) - rstart[r];
}

__global__ void k_run_head(const uint32_t* __restrict__ list, uint32_t nlong,
                           const uint32_t* __restrict__ first_run,
                           const uint32_t* __restrict__ nruns, uint4* __restrict__ head) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= nlong) return;
    const uint32_t r0 = first_run[i];
    const uint32_t r1 = (i + 1 < nlong) ? first_run[i + 1] : *nruns;
    uint4 e = head[list[i]];
    e.z = r0;
    e.w = r1 - r0;
    head[list[i]] = e;
}

// per-bin tallies -> two count arrays
__global__ void k_split_tally(const uint2* __restrict__ tally, uint32_t bins,
                              uint32_t* __restrict__ cnt, uint32_t* __restrict__ len) {
    const uint32_t g = blockIdx.x * kThreads + threadIdx.x;
    if (g < bins) {
        const uint2 t = tally[g];
        cnt[g] = t.x;
        len[g] = t.y;
    }
}

// Long buckets of every bin with any, ascending, at the bin's slot range.
__global__ __launch_bounds__(kThreads) void k_list_long(const uint32_t* __restrict__ off,
                                                        uint32_t V, uint32_t k, uint32_t bins,
                                                        const uint2* __restrict__ tally,
                                                        const uint32_t* __restrict__ pre,
                                                        uint32_t* __restrict__ list) {
    __shared__ uint32_t tmp[kThreads / kWave + 1];
    const uint32_t NB = 1u << k;
    for (uint32_t g = blockIdx.x; g < bins; g += gridDim.x) {
        if (tally[g].x == 0) continue;  // uniform across the workgroup
        const uint32_t v0 = g << k, nb = (V - v0 < NB) ? V - v0 : NB;
        uint32_t at = pre[g];
        for (uint32_t c0 = 0; c0 < nb; c0 += kThreads) {
            const uint32_t v = c0 + threadIdx.x;
            const uint32_t f = (v < nb && off[v0 + v + 1] - off[v0 + v] > kRunBucket) ? 1u : 0u;
            uint32_t all;
            const uint32_t r = block_excl_scan<kThreads>(f, tmp, &all);
            if (f) list[at + r] = v0 + v;
            at += all;
        }
    }
}

size_t sort_tmp_bytes(uint32_t total, int key_bits) {
    size_t a = 0, b = 0;
    (void)rocprim::radix_sort_pairs((void*)nullptr, a, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                    (uint32_t*)nullptr, (uint32_t*)nullptr, total, 0, 64);
    if (key_bits == 64)
        (void)rocprim::radix_sort_pairs((void*)nullptr, b, (uint32_t*)nullptr,
                                        (uint32_t*)nullptr, (uint32_t*)nullptr,
                                        (uint32_t*)nullptr, total, 0, 32);
    return a > b ? a : b;
}

struct RunsWs {
    uint32_t *len, *base, *pos, *pos_s, *idx, *idx_s, *seg, *seg2, *seg2_s, *ord, *ord_s;
    uint64_t *sk, *sk_s;
    uint32_t *flag, *rid, *rstart, *first_run;
    void* scan_ws;
    void* sort_tmp;
    size_t sort_bytes;
};

size_t layout_runs(void* ws, uint64_t nlong, uint64_t total, int key_bits, RunsWs* w) {
    Carver c(ws);
    RunsWs t{};
    t.len = c.take<uint32_t>(nlong + 1);
    t.base = c.take<uint32_t>(nlong + 1);
    t.sk = c.take<uint64_t>(total);
    t.sk_s = c.take<uint64_t>(total);
    t.pos = c.take<uint32_t>(total);
    t.pos_s = c.take<uint32_t>(total);
    if (key_bits == 64) {
        t.idx = c.take<uint32_t>(total);
        t.idx_s = c.take<uint32_t>(total);
        t.seg = c.take<uint32_t>(total);
        t.seg2 = c.take<uint32_t>(total);
        t.seg2_s = c.take<uint32_t>(total);
        t.ord = c.take<uint32_t>(total);
        t.ord_s = c.take<uint32_t>(total);
    }
    t.flag = c.take<uint32_t>(total);
    t.rid = c.take<uint32_t>(total + 1);
    t.rstart = c.take<uint32_t>(total);
    t.first_run = c.take<uint32_t>(nlong + 1);
    const uint64_t sn = total > nlong ? total : nlong;
    t.scan_ws = c.take<char>(scan_ws_bytes(sn));
    t.sort_bytes = sort_tmp_bytes((uint32_t)total, key_bits);
    t.sort_tmp = c.take<char>(t.sort_bytes);
    if (w) *w = t;
    return c.off + 256;
}

}  // namespace

size_t tally_ws_bytes(uint32_t bins) {
    return 2 * align_up(((size_t)bins + 1) * 4, 256) + scan_ws_bytes(bins) + 512;
}

hipError_t scan_tally(const uint2* tally, uint32_t bins, uint32_t* pre_cnt, uint32_t* pre_len,
                      void* ws, hipStream_t s) {
    Carver c(ws);
    uint32_t* cnt = c.take<uint32_t>((size_t)bins + 1);
    uint32_t* len = c.take<uint32_t>((size_t)bins + 1);
    void* sws = c.take<char>(scan_ws_bytes(bins));
    hipLaunchKernelGGL(k_split_tally, dim3(blocks_for(bins)), dim3(kThreads), 0, s, tally, bins,
                       cnt, len);
    HG_TRY(hipGetLastError());
    HG_TRY(scan_excl<uint32_t>(cnt, bins, pre_cnt, nullptr, sws, s));
    return scan_excl<uint32_t>(len, bins, pre_len, nullptr, sws, s);
}

hipError_t list_long_buckets(const uint32_t* offsets, uint64_t V, uint32_t k, uint32_t bins,
                             const uint2* tally, const uint32_t* pre_cnt, uint32_t* long_list,
                             hipStream_t s) {
    const uint32_t grid = bins < 16384 ? bins : 16384;
    hipLaunchKernelGGL(k_list_long, dim3(grid ? grid : 1), dim3(kThreads), 0, s, offsets,
                       (uint32_t)V, k, bins, tally, pre_cnt, long_list);
    return hipGetLastError();
}

size_t runs_ws_bytes(uint64_t nlong, uint64_t total, int key_bits) {
    return layout_runs(nullptr, nlong, total, key_bits, nullptr);
}

template <typename Key>
hipError_t run_key_runs(const uint32_t* offsets, const uint32_t* ids, const Key* ekeys,
                        const uint32_t* long_list, uint32_t nlong, uint32_t total, uint4* head,
                        const RunsDev& r, void* ws, hipStream_t s) {
    if (nlong == 0 || total == 0) return hipSuccess;
    RunsWs w;
    layout_runs(ws, nlong, total, sizeof(Key) * 8, &w);
    HG_PROF("runs_build", s);
    hipLaunchKernelGGL(k_long_len, dim3(blocks_for(nlong)), dim3(kThreads), 0, s, offsets,
                       long_list, nlong, w.len);
    HG_TRY(hipGetLastError());
    HG_TRY(scan_excl<uint32_t>(w.len, nlong, w.base, nullptr, w.scan_ws, s));
    Sorted<Key> sv{};
    size_t tmp = w.sort_bytes;
    if constexpr (sizeof(Key) == 4) {
        hipLaunchKernelGGL(k_gather32, dim3(blocks_for(total)), dim3(kThreads), 0, s, offsets,
                           long_list, (const uint32_t*)w.base, nlong, total, ekeys, w.sk, w.pos);
        HG_TRY(hipGetLastError());
        HG_TRY(rocprim::radix_sort_pairs(w.sort_tmp, tmp, w.sk, w.sk_s, w.pos, w.pos_s, total, 0u,
                                         32u + bits_for(nlong), s));
        sv.comp = w.sk_s;
        sv.spos = w.pos_s;
    } else {
        hipLaunchKernelGGL(k_gather64, dim3(blocks_for(total)), dim3(kThreads), 0, s, offsets,
                           long_list, (const uint32_t*)w.base, nlong, total, ekeys, w.sk, w.idx,
                           w.seg, w.pos);
        HG_TRY(hipGetLastError());
        // by key, then stably by list index
        HG_TRY(rocprim::radix_sort_pairs(w.sort_tmp, tmp, w.sk, w.sk_s, w.idx, w.idx_s, total,
                                         0u, 64u, s));
        hipLaunchKernelGGL(k_seg_of, dim3(blocks_for(total)), dim3(kThreads), 0, s,
                           (const uint32_t*)w.idx_s, (const uint32_t*)w.seg, total, w.seg2,
                           w.ord);
        HG_TRY(hipGetLastError());
        tmp = w.sort_bytes;
        const uint32_t sb = bits_for(nlong);
        if (sb) {
            HG_TRY(rocprim::radix_sort_pairs(w.sort_tmp, tmp, w.seg2, w.seg2_s, w.ord, w.ord_s,
                                             total, 0u, sb, s));
            sv.sseg = w.seg2_s;
            sv.ord = w.ord_s;
        } else {
            sv.sseg = w.seg2;
            sv.ord = w.ord;
        }
        // ord[j] indexes the key-sorted arrays: key sk_s, position pos[idx_s]
        hipLaunchKernelGGL(k_seg_of, dim3(blocks_for(total)), dim3(kThreads), 0, s,
                           (const uint32_t*)w.idx_s, (const uint32_t*)w.pos, total, w.pos_s,
                           w.idx);  // pos_s[t] = pos[idx_s[t]]; idx reused as scratch
        HG_TRY(hipGetLastError());
        sv.skey = (const Key*)w.sk_s;
        sv.spos = w.pos_s;
    }
    hipLaunchKernelGGL(k_run_flags<Key>, dim3(blocks_for(total)), dim3(kThreads), 0, s, sv, total,
                       w.flag);
    HG_TRY(hipGetLastError());
    HG_TRY(scan_excl<uint32_t>(w.flag, total, w.rid, nullptr, w.scan_ws, s));
    hipLaunchKernelGGL(k_run_emit<Key>, dim3(blocks_for(total)), dim3(kThreads), 0, s, sv, total,
                       (const uint32_t*)w.flag, (const uint32_t*)w.rid, offsets, long_list,
                       (const uint32_t*)w.base, ids, (Key*)r.run_key, r.run_pos, w.rstart,
                       w.first_run, r.kperm);
    HG_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_run_cnt, dim3(blocks_for(total)), dim3(kThreads), 0, s,
                       (const uint32_t*)w.rstart, (const uint32_t*)(w.rid + total), total,
                       r.run_cnt);
    HG_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_run_head, dim3(blocks_for(nlong)), dim3(kThreads), 0, s, long_list,
                       nlong, (const uint32_t*)w.first_run, (const uint32_t*)(w.rid + total),
                       head);
    return hipGetLastError();
}

template hipError_t run_key_runs<uint32_t>(const uint32_t*, const uint32_t*, const uint32_t*,
                                           const uint32_t*, uint32_t, uint32_t, uint4*,
                                           const RunsDev&, void*, hipStream_t);
template hipError_t run_key_runs<uint64_t>(const uint32_t*, const uint32_t*, const uint64_t*,
                                           const uint32_t*, uint32_t, uint32_t, uint4*,
                                           const RunsDev&, void*, hipStream_t);

}  // namespace hg
