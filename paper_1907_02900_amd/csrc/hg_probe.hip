// Probing a HashGraph (Sec. 3.4).
//
// HashGraph-Probe-Standard: each query is hashed with Eq. 1, the bucket's
// segment [offsets[h], offsets[h+1]) of the edge array is scanned, and every
// entry with an equal key is counted (all instances, not the first).  When
// the V2 build wrote the per-bucket probe index, the segment bounds and the
// bucket's first keys come from one 16-byte entry instead, so a query into a
// bucket of at most two 32-bit keys (one 64-bit key) costs one random read.  Each
// thread owns several queries (coalesced, strided by the block) and issues
// all their offset loads before scanning, to keep many random reads in
// flight.  Pairs are written in a second pass at positions given by an
// exclusive scan of the counts, so pairs are grouped by query id.
//
// HashGraph-Probe-New (Alg. 3): both inputs are built into HashGraphs with the
// same hash and V, and bucket x of A is intersected with bucket x of B for
// every x.  B's edges are walked in edge order, so the buckets of A are read
// in increasing order (streaming, cache-friendly) instead of at random.
#include "hg_internal.h"

namespace hg {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeItems = 8;

// Entries of ekeys[lo, hi) equal to q.  Past the first few keys the scan
// reads 16 bytes at a time (aligned), so a medium bucket costs a few wide
// loads instead of one load per key.
template <typename Key>
__device__ __forceinline__ uint32_t count_in_bucket(const Key* __restrict__ ekeys, uint32_t lo,
                                                    uint32_t hi, Key q) {
    constexpr uint32_t V = 16 / sizeof(Key);  // keys per 16-byte load
    uint32_t c = 0;
    uint32_t p = lo;
    if (hi - lo > 2 * V) {
        for (; p % V; ++p) c += (ekeys[p] == q) ? 1u : 0u;
        for (; p + V <= hi; p += V) {
            const uint4 w = *reinterpret_cast<const uint4*>(ekeys + p);
            if constexpr (sizeof(Key) == 4) {
                c += (w.x == q) + (w.y == q) + (w.z == q) + (w.w == q);
            } else {
                c += ((((uint64_t)w.y << 32) | w.x) == q) + ((((uint64_t)w.w << 32) | w.z) == q);
            }
        }
    }
    for (; p < hi; ++p) c += (ekeys[p] == q) ? 1u : 0u;
    return c;
}

// What a probe index entry holds (x = the bucket's length; see head_entry):
// 32-bit keys: all keys of a bucket of at most three in y, z, w, else the
// start in y, the first key in z and, in w, the number of entries equal to it
// (low 8 bits) and the filter of the bucket's other keys (high 24 bits);
// 64-bit keys: the start in y and in z, w the key of a one-key bucket or the
// filter of a longer bucket's keys.  A bucket longer than kRunBucket has its
// key-run summary in z, w instead.
template <typename Key>
struct HeadKeys;

template <>
struct HeadKeys<uint32_t> {
    static constexpr uint32_t full = 3;  // buckets this short keep every key, no start
    __device__ static bool has_start(uint32_t len) { return len > full; }
    __device__ static uint32_t stored(uint32_t len) { return len <= full ? len : 1u; }
    __device__ static uint32_t key(const uint4& e, uint32_t len, uint32_t i) {
        if (len <= full) return i == 0 ? e.y : (i == 1 ? e.z : e.w);
        return e.z;
    }
};

template <>
struct HeadKeys<uint64_t> {
    __device__ static bool has_start(uint32_t) { return true; }
    __device__ static uint32_t stored(uint32_t len) { return len == 1 ? 1u : 0u; }
    __device__ static uint64_t key(const uint4& e, uint32_t, uint32_t) {
        return (uint64_t)e.z | ((uint64_t)e.w << 32);
    }
};

// Key-run summary of the long buckets (see hg_runs.hip and RunsDev): runs
// of a bucket starting at edge position st are at [st, st + R) of key / end.
template <typename Key>
struct Runs {
    const Key* key;         // distinct keys, ascending inside each long bucket
    const uint32_t* end;    // end of each run's group (offset from the bucket start)
    const uint32_t* kperm;  // ids grouped by key (buckets of several keys)
};

template <typename Key>
Runs<Key> runs_of(const TableDev& t) {
    return Runs<Key>{(const Key*)t.runs.run_key, t.runs.run_end, t.runs.kperm};
}

// Run of q among runs [r0, r0 + d) (keys ascending), or ~0u if q is absent.
template <typename Key>
__device__ __forceinline__ uint32_t find_run(const Key* __restrict__ rk, uint32_t r0, uint32_t d,
                                             Key q) {
    uint32_t lo = r0, hi = r0 + d;  // first run with key >= q
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (rk[mid] < q) lo = mid + 1;
        else hi = mid;
    }
    return (lo < r0 + d && rk[lo] == q) ? lo : ~0u;
}

// Group [*b, *e) (offsets from the bucket start) of q in a long bucket whose
// index entry is e = {len, st, R, key}; false if q is not in the bucket.  A
// bucket of one key (R = 1) is answered from its entry (32-bit keys) or its
// single run key.
template <typename Key>
__device__ __forceinline__ bool run_group(const uint4& e, const Runs<Key>& runs, Key q,
                                          uint32_t* gb, uint32_t* ge) {
    const uint32_t st = e.y, R = e.z;
    if (R == 1) {
        const bool hit = sizeof(Key) == 4 ? (uint32_t)q == e.w : runs.key[st] == q;
        *gb = 0;
        *ge = e.x;
        return hit;
    }
    const uint32_t r = find_run(runs.key, st, R, q);
    if (r == ~0u) return false;
    *gb = r > st ? runs.end[r - 1] : 0u;
    *ge = runs.end[r];
    return true;
}

// Matches of q in a bucket described by its index entry: the keys held in the
// entry are compared directly, the edge array is read only past them; a long
// bucket's entry points at its key runs instead (R = 0: no runs, scanned).
template <typename Key>
__device__ __forceinline__ uint32_t count_with_head(const uint4& e, const Key* __restrict__ ekeys,
                                                    const Runs<Key>& runs, Key q) {
    using HK = HeadKeys<Key>;
    const uint32_t len = e.x;
    if (len > kRunBucket) {
        if (e.z == 0) return count_in_bucket(ekeys, e.y, e.y + len, q);  // runs dropped by an erase
        uint32_t gb, ge;
        return run_group(e, runs, q, &gb, &ge) ? ge - gb : 0u;
    }
    if (sizeof(Key) == 4 && len > HeadKeys<uint32_t>::full) {
        // {len, start, first key, its count | filter}: the first key's
        // matches are counted in the entry; the rest of the bucket is read
        // only when the query is not the first key and its filter bit is set
        // (a clear bit: no other key of the bucket equals q)
        if ((uint32_t)q == e.z) return e.w & 0xffu;
        if (!((e.w >> (8 + filter_bit((uint32_t)q))) & 1u)) return 0u;
        return count_in_bucket(ekeys, e.y + 1, e.y + len, q);
    }
    if (sizeof(Key) == 8 && len > 1) {
        // {len, start, filter of the bucket's keys}: read the bucket only
        // when both of q's filter bits are set
        const uint64_t f = (uint64_t)e.z | ((uint64_t)e.w << 32), b = filter_bits64((uint64_t)q);
        if ((f & b) != b) return 0u;
        return count_in_bucket(ekeys, e.y, e.y + len, q);
    }
    const uint32_t n = HK::stored(len);
    uint32_t c = 0;
#pragma unroll
    for (uint32_t i = 0; i < 3; ++i) c += (i < n && HK::key(e, len, i) == q) ? 1u : 0u;
    if (len > n) c += count_in_bucket(ekeys, e.y + n, e.y + len, q);  // the start is stored
    return c;
}

// For the pairs pass: 0x80 | the mask of the entry's keys equal to q when the
// bucket (1-3 32-bit keys) is held whole in its entry, else 0.
template <typename Key>
__device__ __forceinline__ uint8_t held_code(const uint4& e, Key q) {
    using HK = HeadKeys<uint32_t>;
    const uint32_t len = e.x;
    if (len == 0 || len > HK::full) return 0;
    uint32_t mask = 0;
#pragma unroll
    for (uint32_t i = 0; i < HK::full; ++i)
        mask |= (i < len && HK::key(e, len, i) == (uint32_t)q) ? 1u << i : 0u;
    return (uint8_t)(0x80u | mask);
}

// Probe-Standard counts.  HEAD: each query reads its bucket's 16-byte index
// entry (one random access for buckets of up to three 32-bit keys or one
// 64-bit key); otherwise it reads
// offsets[h], offsets[h+1] and scans the edge array.  xcd_tiles = 0: block b
// takes query tile b; else the grid has 8 * ceil(xcd_tiles / 8) blocks and
// tiles are dealt out by xcd_tile, so that each XCD walks one contiguous run
// of queries (queries grouped by bucket range then read one L2-sized window
// of the index per XCD at a time).  gate (may be null): when *gate == 0 the
// launch probes q_in into counts_in instead, block b taking tile b (the
// grouped probe decides on the device whether its queries were grouped).
template <typename Key, bool HEAD>
__global__ __launch_bounds__(kProbeThreads) void k_probe_count(
    const Key* __restrict__ q, uint64_t m, typename KeyTraits<Key>::Params hp,
    const uint32_t* __restrict__ off, const uint4* __restrict__ head, Runs<Key> runs,
    const Key* __restrict__ ekeys, uint32_t* __restrict__ counts,
    unsigned long long* __restrict__ total, uint8_t* __restrict__ held, uint32_t xcd_tiles,
    const uint32_t* __restrict__ gate, const Key* __restrict__ q_in,
    uint32_t* __restrict__ counts_in) {
    __shared__ uint64_t red[kProbeThreads / kWave + 1];
    uint32_t tile = xcd_tiles ? xcd_tile(blockIdx.x, xcd_tiles) : blockIdx.x;
    if (gate && *gate == 0u) {
        q = q_in;
        counts = counts_in;
        tile = blockIdx.x;
    }
    const uint64_t base = (uint64_t)tile * (kProbeThreads * kProbeItems) + threadIdx.x;
    Key qq[kProbeItems];
    uint4 e[kProbeItems];
#pragma unroll
    for (int r = 0; r < kProbeItems; ++r) {
        const uint64_t j = base + (uint64_t)r * kProbeThreads;
        qq[r] = (j < m) ? q[j] : (Key)0;
    }
#pragma unroll
    for (int r = 0; r < kProbeItems; ++r) {
        const uint64_t j = base + (uint64_t)r * kProbeThreads;
        if (j < m) {
            const uint32_t h = KeyTraits<Key>::bucket(qq[r], hp);
            if (HEAD) {
                e[r] = head[h];
            } else {
                e[r].x = off[h];
                e[r].y = off[h + 1];
            }
        } else {
            e[r] = make_uint4(0u, 0u, 0u, 0u);
        }
    }
    uint64_t sum = 0;
#pragma unroll
    for (int r = 0; r < kProbeItems; ++r) {
        const uint64_t j = base + (uint64_t)r * kProbeThreads;
        const uint32_t c = HEAD ? count_with_head(e[r], ekeys, runs, qq[r])
                                : count_in_bucket(ekeys, e[r].x, e[r].y, qq[r]);
        if (j < m && counts) counts[j] = c;
        if (HEAD && sizeof(Key) == 4 && held && j < m) held[j] = held_code(e[r], qq[r]);
        sum += c;
    }
    if (total) {
        uint64_t all;
        block_excl_scan64<kProbeThreads>(sum, red, &all);
        if (threadIdx.x == 0) total[1 + blockIdx.x] = all;  // reduced by sum_u64
    }
}

template <typename Key, bool HEAD>
__global__ __launch_bounds__(kProbeThreads) void k_probe_pairs(
    const Key* __restrict__ q, uint64_t m, typename KeyTraits<Key>::Params hp,
    const uint32_t* __restrict__ off, const uint4* __restrict__ head, Runs<Key> runs,
    const Key* __restrict__ ekeys, const uint32_t* __restrict__ eids,
    const uint64_t* __restrict__ positions, uint32_t* __restrict__ build_ids,
    uint32_t* __restrict__ probe_ids, const uint8_t* __restrict__ held) {
    using HK = HeadKeys<Key>;
    // as in k_probe_count: every thread first loads the index entries (or
    // offsets) of its kProbeItems queries, so that their random reads overlap;
    // a query whose output range [positions[j], positions[j+1]) is empty has
    // no match and reads nothing more
    const uint64_t base = (uint64_t)blockIdx.x * (kProbeThreads * kProbeItems) + threadIdx.x;
    // (with the counting pass's codes, a query whose bucket is held whole in
    // its entry skips the entry: it knows its matching keys and reads only
    // the bucket's start)
    Key qq[kProbeItems];
    uint32_t hh[kProbeItems];
    uint4 e[kProbeItems];
    uint64_t pend[kProbeItems];
    bool none[kProbeItems];
    uint32_t code[kProbeItems];
#pragma unroll
    for (int r = 0; r < kProbeItems; ++r) {
        const uint64_t j = base + (uint64_t)r * kProbeThreads;
        qq[r] = (j < m) ? q[j] : (Key)0;
        pend[r] = (j < m) ? positions[j + 1] : 0ull;
        none[r] = j >= m || positions[j] == pend[r];
        code[r] = (HEAD && held && j < m) ? held[j] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kProbeItems; ++r) {
        hh[r] = KeyTraits<Key>::bucket(qq[r], hp);
        if (none[r] || code[r]) {
            e[r] = make_uint4(0u, 0u, 0u, 0u);
        } else if (HEAD) {
            e[r] = head[hh[r]];
        } else {
            e[r].x = off[hh[r]];
            e[r].y = off[hh[r] + 1];
        }
    }
    // where each query's bucket starts (a bucket whose keys are all in its
    // entry needs offsets[h], read only when one of those keys matches), and
    // how many leading keys the entry holds; the loads overlap across queries
    uint32_t st[kProbeItems], nn[kProbeItems];
    bool skip[kProbeItems], via_runs[kProbeItems];
#pragma unroll
    for (int r = 0; r < kProbeItems; ++r) {
        const uint4 er = e[r];
        skip[r] = none[r];
        via_runs[r] = false;
        nn[r] = 0;
        st[r] = er.x;
        if (HEAD && !skip[r] && code[r]) {
            st[r] = off[hh[r]];
        } else if (HEAD && !skip[r]) {
            const uint32_t len = er.x;
            const bool longb = len > kRunBucket;
            via_runs[r] = longb && er.z != 0u;
            nn[r] = longb ? 0u : HK::stored(len);
            if (HK::has_start(len)) {
                st[r] = er.y;
            } else {
                bool any = false;
                for (uint32_t i = 0; i < nn[r]; ++i) any |= HK::key(er, len, i) == qq[r];
                skip[r] = !any;
                st[r] = any ? off[hh[r]] : 0u;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kProbeItems; ++r) {
        if (skip[r]) continue;
        const uint64_t j = base + (uint64_t)r * kProbeThreads;
        const Key k = qq[r];
        const uint4 er = e[r];
        uint64_t pos = positions[j];
        if (code[r]) {
#pragma unroll
            for (uint32_t i = 0; i < 3; ++i)
                if (((code[r] >> i) & 1u) && pos < pend[r]) {
                    build_ids[pos] = eids[st[r] + i];
                    probe_ids[pos] = (uint32_t)j;
                    ++pos;
                }
            continue;
        }
        if (via_runs[r]) {
            // the ids of q's group, in bucket order: the edge array's own for
            // a bucket of one key, else its group in kperm
            uint32_t gb, ge;
            if (run_group(er, runs, k, &gb, &ge)) {
                const uint32_t* src = er.z == 1 ? eids + er.y : runs.kperm + er.y;
                for (uint32_t t = gb; t < ge && pos < pend[r]; ++t) {
                    build_ids[pos] = src[t];
                    probe_ids[pos] = (uint32_t)j;
                    ++pos;
                }
            }
            continue;
        }
        const uint32_t start = st[r], len = HEAD ? er.x : er.y - er.x, n = nn[r];
        for (uint32_t p = start; p < start + len && pos < pend[r]; ++p)
            if ((p - start < n ? HK::key(er, len, p - start) : ekeys[p]) == k) {
                build_ids[pos] = eids[p];
                probe_ids[pos] = (uint32_t)j;
                ++pos;
            }
    }
}

// Alg. 3 over B's edges p: count the entries of A's bucket h(key_p) equal to
// key_p.  A and B share hash parameters, so h is recomputed from B's key.
// Matches of k in A's bucket h: a scan, or A's key runs when the bucket is
// long and A has them (a_head not null).
template <typename Key>
__device__ __forceinline__ uint32_t count_in_a(const uint32_t* __restrict__ a_off,
                                               const uint32_t* __restrict__ a_len,
                                               const uint4* __restrict__ a_head,
                                               const Runs<Key>& runs,
                                               const Key* __restrict__ a_keys, uint32_t h,
                                               Key k) {
    const uint32_t lo = a_off[h], hi = a_len ? lo + a_len[h] : a_off[h + 1];
    if (a_head && hi - lo > kRunBucket) {
        const uint4 e = a_head[h];
        uint32_t gb, ge;
        if (e.z != 0) return run_group(e, runs, k, &gb, &ge) ? ge - gb : 0u;
    }
    return count_in_bucket(a_keys, lo, hi, k);
}

// B's stale slots (behind a bucket's live entries after an erase) are skipped:
// they get edge count 0 and write no count by input.
template <typename Key>
__global__ __launch_bounds__(kProbeThreads) void k_intersect_count(
    const uint32_t* __restrict__ a_off, const uint32_t* __restrict__ a_len,
    const uint4* __restrict__ a_head, Runs<Key> runs, const Key* __restrict__ a_keys,
    const uint32_t* __restrict__ b_off, const uint32_t* __restrict__ b_len,
    const Key* __restrict__ b_keys, const uint32_t* __restrict__ b_ids, uint64_t nb,
    typename KeyTraits<Key>::Params hp, uint32_t* __restrict__ edge_counts,
    uint32_t* __restrict__ counts_by_input, unsigned long long* __restrict__ total) {
    __shared__ uint64_t red[kProbeThreads / kWave + 1];
    uint64_t sum = 0;
    const uint64_t base = (uint64_t)blockIdx.x * (kProbeThreads * kProbeItems) + threadIdx.x;
#pragma unroll
    for (int r = 0; r < kProbeItems; ++r) {
        const uint64_t p = base + (uint64_t)r * kProbeThreads;
        if (p < nb) {
            const Key k = b_keys[p];
            const uint32_t h = KeyTraits<Key>::bucket(k, hp);
            if (b_len && p - b_off[h] >= b_len[h]) {
                if (edge_counts) edge_counts[p] = 0;
                continue;
            }
            const uint32_t c = count_in_a(a_off, a_len, a_head, runs, a_keys, h, k);
            if (edge_counts) edge_counts[p] = c;
            if (counts_by_input) counts_by_input[b_ids[p]] = c;
            sum += c;
        }
    }
    if (total) {
        uint64_t all;
        block_excl_scan64<kProbeThreads>(sum, red, &all);
        if (threadIdx.x == 0) total[1 + blockIdx.x] = all;  // reduced by sum_u64
    }
}

template <typename Key>
__global__ __launch_bounds__(kProbeThreads) void k_intersect_pairs(
    const uint32_t* __restrict__ a_off, const uint32_t* __restrict__ a_len,
    const uint4* __restrict__ a_head, Runs<Key> runs, const Key* __restrict__ a_keys,
    const uint32_t* __restrict__ a_ids, const uint32_t* __restrict__ b_off,
    const uint32_t* __restrict__ b_len, const Key* __restrict__ b_keys,
    const uint32_t* __restrict__ b_ids, uint64_t nb, typename KeyTraits<Key>::Params hp,
    const uint64_t* __restrict__ positions, uint32_t* __restrict__ out_a,
    uint32_t* __restrict__ out_b) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (; p < nb; p += st) {
        // an edge whose output range is empty (no match, or a stale slot of
        // B, whose count is 0) reads nothing more
        uint64_t pos = positions[p];
        const uint64_t pend = positions[p + 1];
        if (pos == pend) continue;
        const Key k = b_keys[p];
        const uint32_t h = KeyTraits<Key>::bucket(k, hp);
        if (b_len && p - b_off[h] >= b_len[h]) continue;  // stale slot of B
        const uint32_t lo = a_off[h], hi = a_len ? lo + a_len[h] : a_off[h + 1];
        const uint32_t bid = b_ids[p];
        if (a_head && hi - lo > kRunBucket) {
            const uint4 e = a_head[h];
            if (e.z != 0) {
                uint32_t gb, ge;
                if (run_group(e, runs, k, &gb, &ge)) {
                    const uint32_t* src = e.z == 1 ? a_ids + e.y : runs.kperm + e.y;
                    for (uint32_t t = gb; t < ge && pos < pend; ++t) {
                        out_a[pos] = src[t];
                        out_b[pos] = bid;
                        ++pos;
                    }
                }
                continue;
            }
        }
        for (uint32_t i = lo; i < hi && pos < pend; ++i)
            if (a_keys[i] == k) {
                out_a[pos] = a_ids[i];
                out_b[pos] = bid;
                ++pos;
            }
    }
}

uint32_t grid_for(uint64_t items, uint32_t per_block) {
    uint64_t g = ceil_div(items, per_block);
    return (uint32_t)(g ? g : 1);
}

}  // namespace

size_t probe_ws_bytes(uint64_t m) {
    // counts (m uint32), positions (m+1 uint64), scan workspace
    return align_up(m * 4, 256) + align_up((m + 1) * 8, 256) + scan_ws_bytes(m) + 512;
}

uint64_t probe_total_slots(uint64_t m) {
    // one per block, the grid rounded up to whole XCD rounds (xcd_order)
    return 1 + (m ? 8 * (((uint64_t)grid_for(m, kProbeThreads * kProbeItems) + 7) / 8) : 0);
}

template <typename Key>
hipError_t run_probe_counts(const TableDev& t, const Key* queries, uint64_t m, uint32_t* counts,
                            unsigned long long* d_total, hipStream_t s, uint8_t* held,
                            bool xcd_order, const uint32_t* gate, const Key* q_in,
                            uint32_t* counts_in) {
    if (m == 0) return d_total ? fill_u32((uint32_t*)d_total, 2, 0u, s) : hipSuccess;
    auto hp = KeyTraits<Key>::make(t.V, t.seed);
    const uint32_t tiles = grid_for(m, kProbeThreads * kProbeItems);
    const uint32_t xt = xcd_order ? tiles : 0u;
    const dim3 grid(xcd_order ? 8 * ((tiles + 7) / 8) : tiles);
    {
        HG_PROF("probe_count", s);
        if (t.head)
            hipLaunchKernelGGL((k_probe_count<Key, true>), grid, dim3(kProbeThreads), 0, s,
                               queries, m, hp, t.offsets, t.head, runs_of<Key>(t),
                               (const Key*)t.keys, counts, d_total, held, xt, gate, q_in,
                               counts_in);
        else
            hipLaunchKernelGGL((k_probe_count<Key, false>), grid, dim3(kProbeThreads), 0, s,
                               queries, m, hp, t.offsets, t.head, runs_of<Key>(t),
                               (const Key*)t.keys, counts, d_total, (uint8_t*)nullptr, xt,
                               gate, q_in, counts_in);
    }
    HG_TRY(hipGetLastError());
    return d_total ? sum_u64(d_total + 1, grid.x, d_total, s) : hipSuccess;
}

template <typename Key>
hipError_t run_probe_pairs(const TableDev& t, const Key* queries, uint64_t m,
                           const uint64_t* positions, uint32_t* build_ids, uint32_t* probe_ids,
                           hipStream_t s, const uint8_t* held) {
    if (m == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(t.V, t.seed);
    const uint32_t g = grid_for(m, kProbeThreads * kProbeItems);
    {
        HG_PROF("probe_pairs", s);
        if (t.head)
            hipLaunchKernelGGL((k_probe_pairs<Key, true>), dim3(g), dim3(kProbeThreads), 0, s,
                               queries, m, hp, t.offsets, t.head, runs_of<Key>(t),
                               (const Key*)t.keys, t.ids, positions, build_ids, probe_ids,
                               sizeof(Key) == 4 ? held : nullptr);
        else
            hipLaunchKernelGGL((k_probe_pairs<Key, false>), dim3(g), dim3(kProbeThreads), 0, s,
                               queries, m, hp, t.offsets, t.head, runs_of<Key>(t),
                               (const Key*)t.keys, t.ids, positions, build_ids, probe_ids,
                               (const uint8_t*)nullptr);
    }
    return hipGetLastError();
}

template <typename Key>
hipError_t run_intersect_counts(const TableDev& a, const TableDev& b, uint32_t* edge_counts,
                                uint32_t* counts_by_input, unsigned long long* d_total,
                                hipStream_t s) {
    if (b.n == 0) return d_total ? fill_u32((uint32_t*)d_total, 2, 0u, s) : hipSuccess;
    auto hp = KeyTraits<Key>::make(a.V, a.seed);
    const uint32_t grid = grid_for(b.n, kProbeThreads * kProbeItems);
    {
        HG_PROF("intersect_count", s);
        hipLaunchKernelGGL(k_intersect_count<Key>, dim3(grid),
                           dim3(kProbeThreads), 0, s, a.offsets, a.len, a.head, runs_of<Key>(a),
                           (const Key*)a.keys, b.offsets, b.len, (const Key*)b.keys, b.ids, b.n,
                           hp, edge_counts, counts_by_input, d_total);
    }
    HG_TRY(hipGetLastError());
    return d_total ? sum_u64(d_total + 1, grid, d_total, s) : hipSuccess;
}

template <typename Key>
hipError_t run_intersect_pairs(const TableDev& a, const TableDev& b, const uint64_t* positions,
                               uint32_t* a_ids, uint32_t* b_ids, hipStream_t s) {
    if (b.n == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(a.V, a.seed);
    uint32_t g = grid_for(b.n, kProbeThreads);
    if (g > 8192) g = 8192;
    {
        HG_PROF("intersect_pairs", s);
        hipLaunchKernelGGL(k_intersect_pairs<Key>, dim3(g), dim3(kProbeThreads), 0, s, a.offsets,
                           a.len, a.head, runs_of<Key>(a), (const Key*)a.keys, a.ids, b.offsets,
                           b.len, (const Key*)b.keys, b.ids, b.n, hp, positions, a_ids, b_ids);
    }
    return hipGetLastError();
}

#define HG_PINST(Key)                                                                           \
    template hipError_t run_probe_counts<Key>(const TableDev&, const Key*, uint64_t, uint32_t*, \
                                              unsigned long long*, hipStream_t, uint8_t*, bool,  \
                                              const uint32_t*, const Key*, uint32_t*);           \
    template hipError_t run_probe_pairs<Key>(const TableDev&, const Key*, uint64_t,             \
                                             const uint64_t*, uint32_t*, uint32_t*,             \
                                             hipStream_t, const uint8_t*);                      \
    template hipError_t run_intersect_counts<Key>(const TableDev&, const TableDev&, uint32_t*,  \
                                                  uint32_t*, unsigned long long*, hipStream_t); \
    template hipError_t run_intersect_pairs<Key>(const TableDev&, const TableDev&,              \
                                                 const uint64_t*, uint32_t*, uint32_t*,         \
                                                 hipStream_t);
HG_PINST(uint32_t)
HG_PINST(uint64_t)

}  // namespace hg
