// Internal host-side interface between the C ABI (hg_api.hip) and the kernel
// translation units.  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <atomic>

#include "hg_device.h"

namespace hg {

#define HG_TRY(expr)                        \
    do {                                    \
        hipError_t e__ = (expr);            \
        if (e__ != hipSuccess) return e__;  \
    } while (0)

// Calls f() the first time it is reached with a given device current and
// then never again for that device (kernel attributes such as the dynamic LDS
// limit are set per device).  Two threads arriving together may both call f,
// which must therefore be idempotent; a failed f is tried again next time.
template <typename F>
hipError_t once_per_device(std::atomic<uint64_t>& done, F&& f) {
    int dev = 0;
    HG_TRY(hipGetDevice(&dev));
    const uint64_t bit = dev >= 0 && dev < 64 ? 1ull << dev : 0;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
    HG_TRY(f());
    done.fetch_or(bit, std::memory_order_release);
    return hipSuccess;
}

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint32_t log2_ceil(uint64_t x) {
    uint32_t r = 0;
    while ((1ull << r) < x) ++r;
    return r;
}
inline uint64_t pow2_ceil(uint64_t x) { return 1ull << log2_ceil(x ? x : 1); }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Event-timed launch range (see hg_prof.hip): inactive unless profiling is on.
struct ProfRange {
    const char* name;
    hipStream_t s;
    hipEvent_t e0 = nullptr;
    ProfRange(const char* nm, hipStream_t st);
    ~ProfRange();
    ProfRange(const ProfRange&) = delete;
    ProfRange& operator=(const ProfRange&) = delete;
};
#define HG_PROF_CAT2(a, b) a##b
#define HG_PROF_CAT(a, b) HG_PROF_CAT2(a, b)
#define HG_PROF(name, s) ::hg::ProfRange HG_PROF_CAT(hg_prof_, __LINE__)(name, s)

// The allocator that temporary workspace comes from (hg_set_allocator); both
// functions NULL means hipMallocAsync / hipFreeAsync.
struct WsHook {
    void* (*alloc)(size_t bytes, hipStream_t s, void* ctx) = nullptr;
    void (*free)(void* p, hipStream_t s, void* ctx) = nullptr;
    void* ctx = nullptr;
};
WsHook ws_hook();  // the hook installed now (hg_api.hip)

// Temporary device memory of one call, released at scope exit in stream
// order: work already enqueued on s may still be using it.  The block goes
// back to the allocator that gave it, even if another hook was installed
// meanwhile.
struct Workspace {
    void* p = nullptr;
    hipStream_t s;
    WsHook h{};
    explicit Workspace(hipStream_t st) : s(st) {}
    Workspace(const Workspace&) = delete;
    Workspace& operator=(const Workspace&) = delete;
    hipError_t get(size_t bytes) {
        if (p) return hipErrorInvalidValue;  // one block per object
        if (bytes == 0) bytes = 256;
        h = ws_hook();
        if (!h.alloc) return hipMallocAsync(&p, bytes, s);
        p = h.alloc(bytes, s, h.ctx);
        if (!p) return hipErrorOutOfMemory;
        if ((uintptr_t)p % 256) {  // the carvers and vector loads assume 256-byte blocks
            h.free(p, s, h.ctx);
            p = nullptr;
            return hipErrorInvalidValue;
        }
        return hipSuccess;
    }
    ~Workspace() {
        if (!p) return;
        if (h.alloc)
            h.free(p, s, h.ctx);
        else
            (void)hipFreeAsync(p, s);
    }
};

// A bump allocator over one workspace buffer (sizes first, then pointers).
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T>
    T* take(size_t count) {
        off = align_up(off, 256);
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// ---- partition geometry shared by the V2 kernels --------------------------
constexpr int kPartThreads = 256;
constexpr int kPartItems = 16;
constexpr uint32_t kPartTile = kPartThreads * kPartItems;  // entries per tile
constexpr int kLocalThreads = 512;
// Keys per thread a bin held in LDS may have, and the bin's capacity: 9 for
// 32-bit keys (4608 keys, bins planned at about 4096); 6 for 64-bit keys
// (3072 keys, bins planned at about 2048, so that a bin's LDS leaves room for
// more workgroups per CU).
template <typename Key>
constexpr int light_items() { return sizeof(Key) == 8 ? 6 : 9; }
template <typename Key>
constexpr uint32_t light_cap() { return kLocalThreads * light_items<Key>(); }
constexpr int kHeavyItems = 8;
constexpr uint32_t kHeavyChunk = kLocalThreads * kHeavyItems;  // chunk of an oversize bin
constexpr uint32_t kSliceKeys = 1u << 17;  // bins above this are split over workgroups
constexpr uint32_t kMaxLocalBits = 12;                          // buckets per bin <= 4096
constexpr uint32_t kMaxDigitBits = 11;                       // partition fan-out <= 2048
constexpr uint32_t kOneTierBits = 9;                         // single partition pass up to 512 bins

// How a V2 build splits the bucket index h (Alg. 2): the low `k` bits pick the
// bucket inside a final bin, the bits above pick the final bin.  The final bin
// index is split into one or two partition digits of b1 (and b2) bits.
struct V2Plan {
    uint32_t k = 0;        // log2 buckets per final bin
    uint32_t bins = 0;     // final bins B2 = ceil(V / 2^k)
    uint32_t tiers = 1;    // partition passes (1 or 2)
    uint32_t b1 = 0, b2 = 0;
    uint64_t n = 0, V = 0;
    uint32_t ntiles1 = 0, nchunks1 = 0, ch1 = 1;
    uint32_t ntiles2_ub = 0, nchunks2_ub = 0, ch2 = 1;
};

V2Plan plan_v2(uint64_t n, uint64_t V, int key_bits, uint32_t bins_hint);

// Workspace bytes needed by a build.
size_t build_ws_bytes(int variant, uint64_t n, uint64_t V, int key_bits, uint32_t bins_hint);

// Scan workspace for `n` inputs.
size_t scan_ws_bytes(uint64_t n);

// Exclusive scan of n uint32 counts into n+1 outputs of OutT.  If `copy` is
// not null it also receives the first n outputs (as uint32).
template <typename OutT>
hipError_t scan_excl(const uint32_t* in, uint64_t n, OutT* out, uint32_t* copy, void* ws,
                     hipStream_t s);

hipError_t fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
// out[ids[p]] = vals[p] for p < n, where ids holds every index of [0, n)
// once; for large n through the V2 partition passes by id and per-bin LDS
// placement (hg_v2.hip).  ws: scatter_perm_ws_bytes(n) bytes.
size_t scatter_perm_ws_bytes(uint64_t n);
hipError_t scatter_perm(const uint32_t* ids, const uint32_t* vals, uint64_t n, uint32_t* out,
                        void* ws, hipStream_t s);
// *out = the longest bucket (max of offsets[b+1] - offsets[b] over b < V).
hipError_t max_bucket_len(const uint32_t* offsets, uint64_t V, uint32_t* out, hipStream_t s);

// Stable LSD radix sort of n (key, value) uint32 pairs by the low `bits` bits
// of the key (hg_sort.hip): ping-pongs between (k0, v0) and (k1, v1); the
// sorted pairs end in (k1, v1) when *in_alt, else in (k0, v0).  ws:
// sort_pairs_ws_bytes(n).
size_t sort_pairs_ws_bytes(uint64_t n);
hipError_t sort_pairs_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint64_t n,
                          uint32_t bits, void* ws, bool* in_alt, hipStream_t s);

// *out = sum of v[0..n) (out outside v).
hipError_t sum_u64(const unsigned long long* v, uint64_t n, unsigned long long* out,
                   hipStream_t s);

// uint64 slots of a probe / intersection total buffer for m queries (or B
// entries): slot 0 receives the total, the others hold per-workgroup sums.
uint64_t probe_total_slots(uint64_t m);

template <typename Key>
hipError_t run_hash(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* out,
                    hipStream_t s);

template <typename Key>
hipError_t run_histogram(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* counts,
                         uint32_t block, bool plain, hipStream_t s);

template <typename Key>
hipError_t run_build_v1(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* offsets,
                        uint32_t* ids, Key* ekeys, void* ws, uint32_t block, bool plain,
                        hipStream_t s);

// ---- probe index -------------------------------------------------------------
// Buckets holding more entries than this get a key-run summary: their distinct
// keys in ascending order, each with its count and the start of its run in a
// key-grouped copy of the bucket's ids.
constexpr uint32_t kRunBucket = 32;

// A 32-bit-key bucket of 4..kRunBucket entries keeps, beside its first key and
// that key's count (low 8 bits of the entry's w), a 24-bit filter of its other
// keys (w's high 24 bits): bit filter_bit(k) is set for every key k of the
// bucket that differs from the first.  A query whose bit is clear matches
// nothing past the first key, so the edge array is not read.  The bit comes
// from a multiplicative hash of the key, not from the bucket hash, so keys of
// one bucket spread over the 24 bits.
constexpr uint32_t kFilterBits = 24;
__host__ __device__ inline uint32_t filter_bit(uint32_t k) {
    return (uint32_t)(((uint64_t)(k * 0x9E3779B1u) * kFilterBits) >> 32);
}

// A 64-bit-key bucket of 2..kRunBucket entries keeps a 64-bit filter of all
// its keys in place of the first key: two bits per key, from the top twelve
// bits of a multiplicative hash.  A query with either bit clear matches none
// of the bucket's keys.
__host__ __device__ inline uint64_t filter_bits64(uint64_t k) {
    const uint64_t x = k * 0x9E3779B97F4A7C15ull;
    return (1ull << (x >> 58)) | (1ull << ((x >> 52) & 63u));
}

// Key-run summary of the long buckets (more than kRunBucket entries): three
// arrays parallel to the edge array.  For a long bucket at edge positions
// [st, st + len) holding R distinct keys, run r < R has the key
// run_key[st + r] (ascending in r) and ends at run_end[st + r] (an offset
// from st: runs are cumulative), and kperm[st .. st + len) lists the bucket's
// ids grouped by key in run order, in bucket order inside each group.  A
// bucket of one repeated key (R = 1) writes no kperm: its ids are the edge
// array's own.  The bucket's probe index entry is {len, st, R, key} with key
// the (32-bit) key when R = 1, else 0; R = 0 marks a long bucket without runs
// (after an erase): probes then scan it.
struct RunsDev {
    void* run_key = nullptr;     // Key[n]
    uint32_t* run_end = nullptr; // [n]
    uint32_t* kperm = nullptr;   // [n]
};

// Long buckets a per-bin kernel leaves to the general pass: bin g lists them
// in gen_list[gen_region(start of bin g, g) ...] and stores their number in
// gen_cnt[g].  A bin of L entries has at most L / (kRunBucket + 1) long
// buckets, so the regions of consecutive bins never overlap and the list
// needs n / (kRunBucket + 1) + bins + 1 entries.
__host__ __device__ inline uint32_t gen_region(uint32_t bin_start, uint32_t g) {
    return bin_start / (kRunBucket + 1) + g;
}
inline uint64_t gen_list_cap(uint64_t n, uint64_t bins) { return n / (kRunBucket + 1) + bins + 1; }

// Where a V2 build writes its probe index (head == null: none) and the
// key-run summary of its long buckets.  k and bins are set by the build.
struct IndexOut {
    uint4* head = nullptr;
    RunsDev runs{};
    uint32_t* gen_list = nullptr;
    uint32_t* gen_cnt = nullptr;  // [bins]
    uint32_t k = 0, bins = 0;
};

// The general pass over the long buckets the per-bin kernels listed (buckets
// of many distinct keys, and every long bucket of the bins too large for
// LDS).  Enqueued after the per-bin build; its work lists live on the device,
// so nothing waits for the host.  ws: runs_ws_bytes(n, bins) bytes; rkeys /
// rids: the build's reorganisation arrays (n entries), free by then and used
// as scratch; ctr: two zeroed counters.
size_t runs_ws_bytes(uint64_t n, uint64_t bins);
template <typename Key>
hipError_t run_key_runs(const uint32_t* offsets, const uint32_t* ids, const Key* ekeys,
                        uint64_t n, const uint32_t* bin_start, uint32_t bins, const IndexOut& ix,
                        Key* rkeys, uint32_t* rids, uint32_t* ctr, void* ws, hipStream_t s);

// ix.head (may be null): V 16-byte probe index entries, one per bucket, and
// the key-run summary of long buckets (IndexOut).  stable: ids ascend inside
// every bucket (otherwise their order there is unspecified).
template <typename Key>
hipError_t run_build_v2(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* offsets,
                        uint32_t* ids, Key* ekeys, IndexOut& ix, void* ws,
                        uint32_t bins_hint, bool stable, hipStream_t s);

// ---- probing ---------------------------------------------------------------
struct TableDev {
    const uint32_t* offsets;
    const uint32_t* ids;
    const void* keys;
    uint64_t n, V, seed;
    const uint4* head = nullptr;  // per-bucket probe index, when the build wrote one
    RunsDev runs{};               // key-run summary of long buckets (with head)
    const uint32_t* len = nullptr;  // live entries per bucket, after an erase (n = slots)
};

// ---- erasing keys ----------------------------------------------------------
// len[h] = offsets[h+1] - offsets[h]
hipError_t init_lengths(const uint32_t* offsets, uint64_t V, uint32_t* len, hipStream_t s);

// Remove every live entry whose key is one of del[0 .. m); dead and touched
// are zeroed byte arrays of t.n and t.V entries (left zeroed); head is the
// table's probe index; *d_removed (device, zeroed) gets the number removed.
template <typename Key>
hipError_t run_erase(const TableDev& t, uint32_t* len, uint8_t* dead, uint8_t* touched,
                     uint4* head, const Key* del, uint64_t m, unsigned long long* d_removed,
                     hipStream_t s);

// Compacted ids / keys of the live entries at new_off (the exclusive scan of
// len); either output may be null.
template <typename Key>
hipError_t run_export_live(const TableDev& t, const uint32_t* len, const uint32_t* new_off,
                           uint32_t* out_ids, Key* out_keys, hipStream_t s);

size_t probe_ws_bytes(uint64_t m);

// counts (may be null) and/or the total (may be null: else a buffer of
// probe_total_slots(m) uint64, the total lands in slot 0).  held (may be
// null; 32-bit keys with the probe index): per query, 0x80 | the mask of the
// matching keys when its bucket is held whole in its index entry, else 0 --
// what the pairs pass needs instead of that entry.
// xcd_order: query tiles are dealt out per XCD (xcd_tile), for queries that
// are grouped by bucket range.  gate (device, may be null): when *gate == 0
// the launch probes q_in into counts_in in input order instead.
template <typename Key>
hipError_t run_probe_counts(const TableDev& t, const Key* queries, uint64_t m, uint32_t* counts,
                            unsigned long long* d_total, hipStream_t s,
                            uint8_t* held = nullptr, bool xcd_order = false,
                            const uint32_t* gate = nullptr, const Key* q_in = nullptr,
                            uint32_t* counts_in = nullptr);

// The same counts (and total) with the queries first grouped by bucket range
// and the counts put back in input order; ws holds
// probe_grouped_ws_bytes(m, t.V, sizeof(Key)) bytes.  decide: a sample of
// the queries taken on the device first picks input order instead when one
// range would hold more than kGroupSkew times its share of them (skewed
// queries read few index lines, which stay cached anyway); the grouping
// passes then find no tiles and the probe launch reads the queries in place.
size_t probe_grouped_ws_bytes(uint64_t m, uint64_t V, size_t key_size);
template <typename Key>
hipError_t run_probe_grouped(const TableDev& t, const Key* queries, uint64_t m, uint32_t* counts,
                             unsigned long long* d_total, void* ws, hipStream_t s,
                             bool decide = false);

// positions[j] = first pair slot of query j (exclusive scan of counts);
// held: the counting pass's per-query codes, or null.
template <typename Key>
hipError_t run_probe_pairs(const TableDev& t, const Key* queries, uint64_t m,
                           const uint64_t* positions, uint32_t* build_ids, uint32_t* probe_ids,
                           hipStream_t s, const uint8_t* held = nullptr);

// Intersection over b's edges: per-edge counts (edge order) and, optionally,
// counts scattered to b's input order.
template <typename Key>
hipError_t run_intersect_counts(const TableDev& a, const TableDev& b, uint32_t* edge_counts,
                                uint32_t* counts_by_input, unsigned long long* d_total,
                                hipStream_t s);

template <typename Key>
hipError_t run_intersect_pairs(const TableDev& a, const TableDev& b, const uint64_t* positions,
                               uint32_t* a_ids, uint32_t* b_ids, hipStream_t s);

// ---- collections: many small tables built once, intersected many times ----

// Device view of a collection (every pointer device memory).
struct CollDev {
    const uint32_t* set_off;  // S + 1 entry offsets of the sets
    const uint64_t* bb;       // S + 2 bucket bases (bb[S] = bb[S+1] = total buckets)
    const uint32_t* offsets;  // total buckets + 1
    const uint32_t* ids;
    const void* keys;
    uint32_t S;
};

// Sizes decided on the device, read back by coll_plan.
struct CollPlan {
    uint64_t *cw, *cb, *cv;  // S + 2 entries each, in the plan workspace
    uint64_t n, buckets, weight, big_keys, big_buckets;
    bool bad;  // set_off not a valid non-decreasing offset array from 0
};

size_t coll_plan_ws_bytes(uint32_t S);
// bb: S + 2 entries, receives the bucket bases; waits for the device.
hipError_t coll_plan(const uint32_t* set_off, uint32_t S, int shift, void* ws, uint64_t* bb,
                     CollPlan* plan, hipStream_t s);
size_t coll_build_ws_bytes(const CollPlan& p, int key_bits);
template <typename Key>
hipError_t run_coll_build(const Key* keys, const uint32_t* set_off, uint32_t S, uint64_t seed,
                          const uint64_t* bb, const CollPlan& p, void* ws, uint32_t* offsets,
                          uint32_t* ids, Key* ekeys, bool* bad, hipStream_t s);
size_t coll_pairs_ws_bytes(uint64_t Q);
// counts (Q entries) and h_total may be null; *bad when a pair index is out of range.
template <typename Key>
hipError_t run_coll_intersect(const CollDev& a, const CollDev& b, uint64_t seed,
                              const uint32_t* pairs, uint64_t Q, unsigned long long* counts,
                              uint64_t* h_total, void* ws, bool* bad, hipStream_t s);

}  // namespace hg
