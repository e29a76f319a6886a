// Key-run summaries of long buckets: exact probing under skew.
//
// Probe-Standard (Sec. 3.4) scans a query's whole bucket.  When many entries
// share a bucket -- heavy duplication, or Zipf keys where one key holds a
// large share of the input -- every probe of that bucket pays its full
// length, so a skewed join costs as much as the number of matching pairs.
// For each bucket longer than kRunBucket the table therefore also keeps the
// bucket's distinct keys in ascending order, each with the number of entries
// holding it and the start of its run in `kperm`, a copy of the bucket's ids
// grouped by key (ids in bucket order inside each group).  The bucket's probe
// index entry points at its runs.  A probe of a long bucket binary-searches
// the runs; its pairs are the ids of one run.  Counts and pairs are exactly
// those of a scan.
//
// Construction: every final bin of the build tallied its long buckets; a scan
// of the tallies sizes the summary and a per-bin pass lists the long buckets.
// A long bucket is usually one key repeated (duplicates) or dominated by one
// key (skew), so the entries equal to their bucket's first key ("lead" key)
// form a run directly, in bucket order, and only the other entries are
// gathered, sorted by (bucket, key) with a stable device radix sort and cut
// into runs.  The lead run is then slotted in at its place among the bucket's
// sorted runs.
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

// largest i in [lo, hi) with base[i] <= j (base non-decreasing, base[lo] <= j)
__device__ __forceinline__ uint32_t owner_in(const uint32_t* __restrict__ base, uint32_t lo,
                                             uint32_t hi, uint32_t j) {
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Owner (long-bucket list index) of gathered entry j = blockIdx.x * kThreads
// + threadIdx.x: the workgroup finds the owners of its first and last entry
// once, so each thread searches only the few buckets its workgroup spans.
// All threads of the workgroup call it (barrier).
__device__ __forceinline__ uint32_t block_owner(const uint32_t* __restrict__ base,
                                                uint32_t nlong, uint32_t total, uint32_t j,
                                                uint32_t* range) {
    if (threadIdx.x == 0) {
        const uint32_t j0 = blockIdx.x * kThreads;
        const uint32_t j1 = (j0 + kThreads < total ? j0 + kThreads : total) - 1;
        range[0] = owner_in(base, 0, nlong, j0);
        range[1] = owner_in(base, range[0], nlong, j1) + 1;
    }
    __syncthreads();
    return owner_in(base, range[0], range[1], j < total ? j : total - 1);
}

// other[j] = 1 if gathered entry j's key differs from its bucket's lead key.
template <typename Key>
__global__ __launch_bounds__(kThreads) void k_mark_others(
    const uint32_t* __restrict__ off, const uint32_t* __restrict__ list,
    const uint32_t* __restrict__ base, uint32_t nlong, uint32_t total,
    const Key* __restrict__ ekeys, uint32_t* __restrict__ other) {
    __shared__ uint32_t range[2];
    const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t i = block_owner(base, nlong, total, j, range);
    if (j >= total) return;
    const uint32_t s = off[list[i]];
    other[j] = (ekeys[s + (j - base[i])] != ekeys[s]) ? 1u : 0u;
}

// Gather the other entries at their compacted slots: 32-bit keys get one
// 64-bit sort key (list index << 32 | key) and their edge position; 64-bit
// keys their key, slot, list index and edge position (two sort passes).
template <typename Key>
__global__ __launch_bounds__(kThreads) void k_gather_others(
    const uint32_t* __restrict__ off, const uint32_t* __restrict__ list,
    const uint32_t* __restrict__ base, uint32_t nlong, uint32_t total,
    const Key* __restrict__ ekeys, const uint32_t* __restrict__ other,
    const uint32_t* __restrict__ opos, uint64_t* __restrict__ sk, uint32_t* __restrict__ idx,
    uint32_t* __restrict__ seg, uint32_t* __restrict__ pos) {
    __shared__ uint32_t range[2];
    const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t i = block_owner(base, nlong, total, j, range);
    if (j >= total || !other[j]) return;
    const uint32_t t = opos[j];
    const uint32_t p = off[list[i]] + (j - base[i]);
    pos[t] = p;
    if constexpr (sizeof(Key) == 4) {
        sk[t] = ((uint64_t)i << 32) | ekeys[p];
    } else {
        sk[t] = ekeys[p];
        idx[t] = t;
        seg[t] = i;
    }
}

// after the key sort of 64-bit keys: out[u] = val[idx[u]], ord[u] = u
__global__ void k_take(const uint32_t* __restrict__ idx, const uint32_t* __restrict__ val,
                       uint32_t total, uint32_t* __restrict__ out, uint32_t* __restrict__ ord) {
    const uint32_t u = blockIdx.x * kThreads + threadIdx.x;
    if (u >= total) return;
    out[u] = val[idx[u]];
    if (ord) ord[u] = u;
}

// Sorted view of the other entries: entry t has list index, key, edge position.
template <typename Key>
struct Sorted {
    const uint32_t* sseg;  // 64-bit keys: list index by sorted position
    const Key* skey;       // 64-bit keys: key by key-sorted index
    const uint64_t* comp;  // 32-bit keys: (list index << 32 | key)
    const uint32_t* spos;  // edge position (by sorted position / key-sorted index)
    const uint32_t* ord;   // 64-bit keys: sorted position -> key-sorted index
};

template <typename Key>
__device__ __forceinline__ void sorted_at(const Sorted<Key>& s, uint32_t t, uint32_t& seg, Key& k,
                                          uint32_t& p) {
    if constexpr (sizeof(Key) == 4) {
        const uint64_t c = s.comp[t];
        seg = (uint32_t)(c >> 32);
        k = (Key)(uint32_t)c;
        p = s.spos[t];
    } else {
        const uint32_t u = s.ord[t];
        seg = s.sseg[t];
        k = s.skey[u];
        p = s.spos[u];
    }
}

template <typename Key>
__global__ void k_run_flags(Sorted<Key> s, uint32_t total, uint32_t* __restrict__ flag) {
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= total) return;
    uint32_t seg, p;
    Key k;
    sorted_at(s, t, seg, k, p);
    uint32_t f = 1;
    if (t) {
        uint32_t seg0, p0;
        Key k0;
        sorted_at(s, t - 1, seg0, k0, p0);
        f = (seg0 != seg || k0 != k) ? 1u : 0u;
    }
    flag[t] = f;
}

// Per long bucket: its first edge, lead-run size, first other entry in sorted
// order, others below the lead key, first run, runs below the lead key.
struct BucketRuns {
    uint32_t start, lead_cnt, obase, nless, rbase, nrless;
};

// One thread per long bucket: place the lead run among the bucket's runs and
// point the index entry at them.
template <typename Key>
__global__ void k_bucket_runs(const uint32_t* __restrict__ off, const uint32_t* __restrict__ list,
                              const uint32_t* __restrict__ base, uint32_t nlong,
                              const uint32_t* __restrict__ opos, const uint32_t* __restrict__ rid,
                              Sorted<Key> s, const Key* __restrict__ ekeys,
                              BucketRuns* __restrict__ br, Key* __restrict__ run_key,
                              uint32_t* __restrict__ run_cnt, uint32_t* __restrict__ run_pos,
                              uint4* __restrict__ head) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= nlong) return;
    const uint32_t b = list[i];
    const uint32_t st = off[b], len = off[b + 1] - st;
    const uint32_t o0 = opos[base[i]], o1 = opos[base[i + 1]];
    const Key lead = ekeys[st];
    // others of this bucket below the lead key (they are sorted by key)
    uint32_t lo = o0, hi = o1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        uint32_t sg, p;
        Key k;
        sorted_at(s, mid, sg, k, p);
        if (k < lead) lo = mid + 1;
        else hi = mid;
    }
    BucketRuns r;
    r.start = st;
    r.lead_cnt = len - (o1 - o0);
    r.obase = o0;
    r.nless = lo - o0;
    r.rbase = i + rid[o0];  // a lead run per earlier bucket, plus their other runs
    r.nrless = rid[lo] - rid[o0];
    br[i] = r;
    const uint32_t slot = r.rbase + r.nrless;
    run_key[slot] = lead;
    run_cnt[slot] = r.lead_cnt;
    run_pos[slot] = st + r.nless;
    uint4 e = head[b];
    e.z = r.rbase;
    e.w = (rid[o1] - rid[o0]) + 1;
    head[b] = e;
}

// Other entries: their kperm slots, and the runs they start.
template <typename Key>
__global__ void k_emit_others(Sorted<Key> s, uint32_t nother, const uint32_t* __restrict__ flag,
                              const uint32_t* __restrict__ rid,
                              const BucketRuns* __restrict__ br, const uint32_t* __restrict__ ids,
                              Key* __restrict__ run_key, uint32_t* __restrict__ run_pos,
                              uint32_t* __restrict__ rstart, uint32_t* __restrict__ rslot,
                              uint32_t* __restrict__ kperm) {
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= nother) return;
    uint32_t seg, p;
    Key k;
    sorted_at(s, t, seg, k, p);
    const BucketRuns r = br[seg];
    const uint32_t lt = t - r.obase;
    const bool above = lt >= r.nless;  // key above the lead key
    const uint32_t at = r.start + lt + (above ? r.lead_cnt : 0u);
    kperm[at] = ids[p];
    if (flag[t]) {
        const uint32_t g = rid[t];  // index among all other runs
        const uint32_t slot = r.rbase + (g - rid[r.obase]) + (above ? 1u : 0u);
        run_key[slot] = k;
        run_pos[slot] = at;
        rstart[g] = t;
        rslot[g] = slot;
    }
}

// counts of the other runs (runs never cross buckets); *nruns other runs
__global__ void k_other_cnt(const uint32_t* __restrict__ rstart,
                            const uint32_t* __restrict__ rslot, const uint32_t* __restrict__ nruns,
                            uint32_t nother, uint32_t* __restrict__ run_cnt) {
    const uint32_t g = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t R = *nruns;
    if (g >= R) return;
    run_cnt[rslot[g]] = ((g + 1 < R) ? rstart[g + 1] : nother) - rstart[g];
}

// Lead-key entries: kperm slots in bucket order, after the bucket's lower others.
__global__ __launch_bounds__(kThreads) void k_emit_lead(
    const uint32_t* __restrict__ base, uint32_t nlong, uint32_t total,
    const uint32_t* __restrict__ other, const uint32_t* __restrict__ opos,
    const BucketRuns* __restrict__ br, const uint32_t* __restrict__ ids,
    uint32_t* __restrict__ kperm) {
    __shared__ uint32_t range[2];
    const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t i = block_owner(base, nlong, total, j, range);
    if (j >= total || other[j]) return;
    const BucketRuns r = br[i];
    const uint32_t lj = j - base[i];                 // position in the bucket
    const uint32_t rank = lj - (opos[j] - r.obase);  // lead entries before it
    kperm[r.start + r.nless + rank] = ids[r.start + lj];
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
    uint32_t *len, *base, *other, *opos;
    uint64_t *sk, *sk_s;
    uint32_t *pos, *pos_s, *idx, *idx_s, *seg, *seg2, *seg2_s, *ord, *ord_s;
    uint32_t *flag, *rid, *rstart, *rslot;
    BucketRuns* br;
    void* scan_ws;
    void* sort_tmp;
    size_t sort_bytes;
};

// Workspace for `total` long-bucket entries (the other entries are at most as
// many).
size_t layout_runs(void* ws, uint64_t nlong, uint64_t total, int key_bits, RunsWs* w) {
    Carver c(ws);
    RunsWs t{};
    t.len = c.take<uint32_t>(nlong + 1);
    t.base = c.take<uint32_t>(nlong + 1);
    t.other = c.take<uint32_t>(total);
    t.opos = c.take<uint32_t>(total + 1);
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
    t.rslot = c.take<uint32_t>(total);
    t.br = c.take<BucketRuns>(nlong);
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
    const dim3 gl(blocks_for(nlong)), gt(blocks_for(total)), th(kThreads);
    hipLaunchKernelGGL(k_long_len, gl, th, 0, s, offsets, long_list, nlong, w.len);
    HG_TRY(hipGetLastError());
    HG_TRY(scan_excl<uint32_t>(w.len, nlong, w.base, nullptr, w.scan_ws, s));
    hipLaunchKernelGGL(k_mark_others<Key>, gt, th, 0, s, offsets, long_list,
                       (const uint32_t*)w.base, nlong, total, ekeys, w.other);
    HG_TRY(hipGetLastError());
    HG_TRY(scan_excl<uint32_t>(w.other, total, w.opos, nullptr, w.scan_ws, s));
    // the sort is sized by the number of other entries
    uint32_t nother = 0;
    HG_TRY(hipMemcpyAsync(&nother, w.opos + total, 4, hipMemcpyDeviceToHost, s));
    HG_TRY(hipStreamSynchronize(s));
    Sorted<Key> sv{};
    if (nother) {
        hipLaunchKernelGGL(k_gather_others<Key>, gt, th, 0, s, offsets, long_list,
                           (const uint32_t*)w.base, nlong, total, ekeys,
                           (const uint32_t*)w.other, (const uint32_t*)w.opos, w.sk, w.idx, w.seg,
                           w.pos);
        HG_TRY(hipGetLastError());
        size_t tmp = w.sort_bytes;
        const dim3 go(blocks_for(nother));
        if constexpr (sizeof(Key) == 4) {
            HG_TRY(rocprim::radix_sort_pairs(w.sort_tmp, tmp, w.sk, w.sk_s, w.pos, w.pos_s,
                                             nother, 0u, 32u + bits_for(nlong), s));
            sv.comp = w.sk_s;
            sv.spos = w.pos_s;
        } else {
            // by key, then stably by list index
            HG_TRY(rocprim::radix_sort_pairs(w.sort_tmp, tmp, w.sk, w.sk_s, w.idx, w.idx_s,
                                             nother, 0u, 64u, s));
            hipLaunchKernelGGL(k_take, go, th, 0, s, (const uint32_t*)w.idx_s,
                               (const uint32_t*)w.seg, nother, w.seg2, w.ord);
            HG_TRY(hipGetLastError());
            const uint32_t sb = bits_for(nlong);
            tmp = w.sort_bytes;
            if (sb) {
                HG_TRY(rocprim::radix_sort_pairs(w.sort_tmp, tmp, w.seg2, w.seg2_s, w.ord,
                                                 w.ord_s, nother, 0u, sb, s));
                sv.sseg = w.seg2_s;
                sv.ord = w.ord_s;
            } else {
                sv.sseg = w.seg2;
                sv.ord = w.ord;
            }
            // edge position of each key-sorted entry
            hipLaunchKernelGGL(k_take, go, th, 0, s, (const uint32_t*)w.idx_s,
                               (const uint32_t*)w.pos, nother, w.pos_s, (uint32_t*)nullptr);
            HG_TRY(hipGetLastError());
            sv.skey = (const Key*)w.sk_s;
            sv.spos = w.pos_s;
        }
        hipLaunchKernelGGL(k_run_flags<Key>, go, th, 0, s, sv, nother, w.flag);
        HG_TRY(hipGetLastError());
    }
    HG_TRY(scan_excl<uint32_t>(w.flag, nother, w.rid, nullptr, w.scan_ws, s));
    hipLaunchKernelGGL(k_bucket_runs<Key>, gl, th, 0, s, offsets, long_list,
                       (const uint32_t*)w.base, nlong, (const uint32_t*)w.opos,
                       (const uint32_t*)w.rid, sv, ekeys, w.br, (Key*)r.run_key, r.run_cnt,
                       r.run_pos, head);
    HG_TRY(hipGetLastError());
    if (nother) {
        const dim3 go(blocks_for(nother));
        hipLaunchKernelGGL(k_emit_others<Key>, go, th, 0, s, sv, nother, (const uint32_t*)w.flag,
                           (const uint32_t*)w.rid, (const BucketRuns*)w.br, ids, (Key*)r.run_key,
                           r.run_pos, w.rstart, w.rslot, r.kperm);
        HG_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_other_cnt, go, th, 0, s, (const uint32_t*)w.rstart,
                           (const uint32_t*)w.rslot, (const uint32_t*)(w.rid + nother), nother,
                           r.run_cnt);
        HG_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_emit_lead, gt, th, 0, s, (const uint32_t*)w.base, nlong, total,
                       (const uint32_t*)w.other, (const uint32_t*)w.opos, (const BucketRuns*)w.br,
                       ids, r.kperm);
    return hipGetLastError();
}

template hipError_t run_key_runs<uint32_t>(const uint32_t*, const uint32_t*, const uint32_t*,
                                           const uint32_t*, uint32_t, uint32_t, uint4*,
                                           const RunsDev&, void*, hipStream_t);
template hipError_t run_key_runs<uint64_t>(const uint32_t*, const uint32_t*, const uint64_t*,
                                           const uint32_t*, uint32_t, uint32_t, uint4*,
                                           const RunsDev&, void*, hipStream_t);

}  // namespace hg
