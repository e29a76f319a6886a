// C ABI of libhashgraph.so (declared in include/hashgraph.h).
//
// Host-side validation, table objects, workspace handling and dispatch to the
// kernels.  Nothing here computes on the CPU: every step of the path runs in
// the HIP kernels of hg_build.hip, hg_scan.hip and hg_probe.hip.
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "hashgraph.h"
#include "hg_internal.h"

using namespace hg;

namespace {
std::mutex g_hook_mu;
WsHook g_hook;  // guarded by g_hook_mu
}  // namespace

WsHook hg::ws_hook() {
    std::lock_guard<std::mutex> lock(g_hook_mu);
    return g_hook;
}

struct hg_table {
    int key_bits = 32;
    int variant = 0;
    uint64_t n = 0, V = 0, seed = 0;
    uint64_t n_cap = 0, V_cap = 0;
    uint32_t* offsets = nullptr;
    uint32_t* ids = nullptr;
    void* keys = nullptr;
    uint4* head = nullptr;  // V_cap per-bucket probe index entries
    bool has_head = false;  // the last build wrote head
    RunsDev runs{};         // key runs of long buckets: n_cap entries per array
    // erasing keys: live entries per bucket, scratch flags, live entry count
    uint32_t* len = nullptr;   // [V_cap]
    uint8_t* dead = nullptr;   // [n_cap]
    uint8_t* touched = nullptr;  // [V_cap]
    bool has_len = false;
    uint64_t live = 0;
    void* ws = nullptr;  // workspace kept for rebuilds (hg_table_create only)
    size_t ws_bytes = 0;
    uint64_t bytes = 0;
};

namespace {

constexpr uint64_t kU32Max = 0xffffffffull;

hg_status from_hip(hipError_t e) {
    if (e == hipSuccess) return HG_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return HG_ERR_OOM;
    if (e == hipErrorInvalidValue) return HG_ERR_INVALID_ARG;
    return HG_ERR_DEVICE;
}

#define HG_CALL(expr)                          \
    do {                                       \
        hipError_t e__ = (expr);               \
        if (e__ != hipSuccess) return from_hip(e__); \
    } while (0)

hg_status device_ready() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return HG_ERR_DEVICE;
    return HG_OK;
}

bool valid_kb(int kb) { return kb == 32 || kb == 64; }
bool valid_range(uint64_t V) { return V >= 1 && V <= kU32Max; }
size_t key_size(int kb) { return kb == 64 ? 8 : 4; }

hg_status read_u64(const uint64_t* d, uint64_t* h, hipStream_t s) {
    HG_CALL(hipMemcpyAsync(h, d, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HG_CALL(hipStreamSynchronize(s));
    return HG_OK;
}

#define HG_CALL_ST(expr)                     \
    do {                                     \
        hg_status st__ = (expr);             \
        if (st__ != HG_OK) return st__;      \
    } while (0)

// The probe index (16 bytes per bucket of the range capacity) and the key-run
// arrays of long buckets (sized for the worst case: every entry in a long
// bucket), allocated once per table.
hg_status ensure_index(hg_table* t) {
    if (t->head) return HG_OK;
    const size_t nc = t->n_cap ? t->n_cap : 1;
    const size_t ks = key_size(t->key_bits);
    HG_CALL(hipMalloc((void**)&t->head, t->V_cap * sizeof(uint4)));
    HG_CALL(hipMalloc(&t->runs.run_key, nc * ks));
    HG_CALL(hipMalloc((void**)&t->runs.run_end, nc * 4));
    HG_CALL(hipMalloc((void**)&t->runs.kperm, nc * 4));
    t->bytes += t->V_cap * sizeof(uint4) + nc * (ks + 8);
    return HG_OK;
}

hg_status build_into(hg_table* t, const void* keys, uint64_t n, uint64_t V, uint64_t seed,
                     const hg_build_opts* opts, hipStream_t s) {
    int variant = opts ? opts->variant : HG_VARIANT_AUTO;
    if (variant == HG_VARIANT_AUTO) variant = HG_VARIANT_V2;
    if (variant != HG_VARIANT_V1 && variant != HG_VARIANT_V2) return HG_ERR_INVALID_ARG;
    const int stable = opts ? opts->stable : 0;
    if (stable && variant == HG_VARIANT_V1) return HG_ERR_INVALID_ARG;
    const uint32_t bins = opts ? opts->bins : 0;
    const uint32_t block = opts ? opts->block : 0;
    const bool v1_plain = opts && opts->v1_plain;
    const bool want_head = variant == HG_VARIANT_V2 && !(opts && opts->no_index);
    const bool any_order = opts && opts->any_order;
    if (any_order && stable) return HG_ERR_INVALID_ARG;
    if (block && (block % 64 || block > 1024)) return HG_ERR_INVALID_ARG;
    if (bins && bins > V) return HG_ERR_INVALID_ARG;

    const size_t need = build_ws_bytes(variant, n, V, t->key_bits, bins);
    Workspace tmp(s);
    void* ws = t->ws;
    if (!ws || t->ws_bytes < need) {
        HG_CALL(tmp.get(need));
        ws = tmp.p;
    }
    if (want_head) HG_CALL_ST(ensure_index(t));
    IndexOut ix{};
    if (want_head) {
        ix.head = t->head;
        ix.runs = t->runs;
    }
    hipError_t e;
    if (t->key_bits == 32) {
        e = variant == HG_VARIANT_V1
                ? run_build_v1<uint32_t>((const uint32_t*)keys, n, V, seed, t->offsets, t->ids,
                                         (uint32_t*)t->keys, ws, block, v1_plain, s)
                : run_build_v2<uint32_t>((const uint32_t*)keys, n, V, seed, t->offsets, t->ids,
                                         (uint32_t*)t->keys, ix, ws, bins, !any_order, s);
    } else {
        e = variant == HG_VARIANT_V1
                ? run_build_v1<uint64_t>((const uint64_t*)keys, n, V, seed, t->offsets, t->ids,
                                         (uint64_t*)t->keys, ws, block, v1_plain, s)
                : run_build_v2<uint64_t>((const uint64_t*)keys, n, V, seed, t->offsets, t->ids,
                                         (uint64_t*)t->keys, ix, ws, bins, !any_order, s);
    }
    if (e != hipSuccess) return from_hip(e);
    t->n = n;
    t->V = V;
    t->seed = seed;
    t->variant = variant;
    t->has_head = want_head;
    t->has_len = false;
    t->live = n;
    return HG_OK;
}

hg_status alloc_table(uint64_t n_cap, uint64_t V_cap, int kb, bool with_ws, hg_table** out) {
    hg_table* t = new (std::nothrow) hg_table();
    if (!t) return HG_ERR_OOM;
    t->key_bits = kb;
    t->n_cap = n_cap;
    t->V_cap = V_cap;
    hipError_t e = hipMalloc((void**)&t->offsets, (V_cap + 1) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&t->ids, (n_cap ? n_cap : 1) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&t->keys, (n_cap ? n_cap : 1) * key_size(kb));
    t->bytes = (V_cap + 1) * 4 + (n_cap ? n_cap : 1) * (4 + key_size(kb));
    if (e == hipSuccess && with_ws) {
        size_t w1 = build_ws_bytes(1, n_cap, V_cap, kb, 0);
        size_t w2 = build_ws_bytes(2, n_cap, V_cap, kb, 0);
        t->ws_bytes = w1 > w2 ? w1 : w2;
        e = hipMalloc(&t->ws, t->ws_bytes);
        t->bytes += t->ws_bytes;
    }
    if (e != hipSuccess) {
        hg_table_free(t);
        return from_hip(e);
    }
    if (with_ws) {
        // a table made for rebuilds holds the index too, so that no build allocates
        const hg_status st = ensure_index(t);
        if (st != HG_OK) {
            hg_table_free(t);
            return st;
        }
    }
    *out = t;
    return HG_OK;
}

hg_status check_table_arg(const hg_table* t) { return t ? HG_OK : HG_ERR_INVALID_ARG; }

TableDev dev_view(const hg_table* t) {
    TableDev d;
    d.offsets = t->offsets;
    d.ids = t->ids;
    d.keys = t->keys;
    d.n = t->n;
    d.V = t->V;
    d.seed = t->seed;
    d.head = t->has_head ? t->head : nullptr;
    if (t->has_head) d.runs = t->runs;
    if (t->has_len) d.len = t->len;
    return d;
}

hg_status check_pairs_args(const hg_table* t, const void* d_queries, uint64_t m,
                           const uint32_t* d_build_ids, const uint32_t* d_probe_ids,
                           uint64_t capacity, const uint64_t* h_total) {
    if (check_table_arg(t) != HG_OK || m > kU32Max || (m && !d_queries) || !h_total)
        return HG_ERR_INVALID_ARG;
    if (capacity && (!d_build_ids || !d_probe_ids)) return HG_ERR_INVALID_ARG;
    if (t->V == 0) return HG_ERR_INVALID_ARG;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    return HG_OK;
}

// Probe-Standard pairs in two passes over a workspace of probe_ws_bytes(m)
// (plus m bytes with `held`): per-query counts, their exclusive scan (64-bit
// positions), the total read back, then each query writes its pairs at its
// position.  With `held` the counting pass also leaves, per query, the
// matching keys of a bucket held whole in its index entry, so the pairs pass
// need not read that entry again.  Every byte of the workspace that is read
// is written first by the same call.
hg_status probe_pairs_into(const hg_table* t, const void* d_queries, uint64_t m,
                           uint32_t* d_build_ids, uint32_t* d_probe_ids, uint64_t capacity,
                           uint64_t* h_total, void* ws, hipStream_t stream, bool with_held) {
    Carver c(ws);
    uint32_t* counts = c.take<uint32_t>(m);
    uint64_t* pos = c.take<uint64_t>(m + 1);
    void* scan_ws = c.take<char>(scan_ws_bytes(m));
    uint8_t* held = with_held && t->key_bits == 32 && t->has_head ? c.take<uint8_t>(m) : nullptr;
    TableDev d = dev_view(t);
    hipError_t e = t->key_bits == 32
                       ? run_probe_counts<uint32_t>(d, (const uint32_t*)d_queries, m, counts, nullptr, stream, held)
                       : run_probe_counts<uint64_t>(d, (const uint64_t*)d_queries, m, counts, nullptr, stream);
    if (e != hipSuccess) return from_hip(e);
    HG_CALL(scan_excl<uint64_t>(counts, m, pos, nullptr, scan_ws, stream));
    hg_status st = read_u64(pos + m, h_total, stream);
    if (st != HG_OK) return st;
    if (*h_total > capacity) return HG_ERR_CAPACITY;
    if (*h_total == 0) return HG_OK;
    e = t->key_bits == 32
            ? run_probe_pairs<uint32_t>(d, (const uint32_t*)d_queries, m, pos, d_build_ids, d_probe_ids, stream, held)
            : run_probe_pairs<uint64_t>(d, (const uint64_t*)d_queries, m, pos, d_build_ids, d_probe_ids, stream);
    if (e != hipSuccess) return from_hip(e);
    HG_CALL(hipStreamSynchronize(stream));
    return HG_OK;
}

// ---- fixed device scratch of the allocation-free entry point -------------
//
// hg_probe_pairs_noalloc's workspace lives in this array, which the code
// object holds on every device the library is loaded on until the process
// ends.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address on the current device comes from
// hipGetSymbolAddress, taken once per device and kept in g_scratch_dev.
constexpr size_t kScratchBytes = (size_t)52 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_dev[64] = {};  // per device ordinal; guarded by g_scratch_mu

// The current device's copy of scratch (looked up on the first call with that
// device current), if it holds `bytes`.
hg_status static_scratch(size_t bytes, void** out) {
    if (bytes > kScratchBytes) return HG_ERR_TOO_LARGE;
    int dev = 0;
    HG_CALL(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return HG_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HG_CALL(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return HG_ERR_DEVICE;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return HG_OK;
}

// ---- single-table autotuner ----------------------------------------------

// skew class of a built table from its longest bucket: 0 = no bucket beyond
// the probe index's short form (32 entries), 1 = none beyond 128, 2 = none
// beyond 512, 3 = none beyond a bin's LDS capacity, 4 = longer (heavy skew)
uint32_t skew_class_of(uint32_t max_len, int kb) {
    if (max_len <= 32) return 0;
    if (max_len <= 128) return 1;
    if (max_len <= 512) return 2;
    return max_len <= (kb == 64 ? 3072u : 4608u) ? 3u : 4u;
}

using TuneKey = std::tuple<uint32_t, uint32_t, int, int, int, int, int, uint32_t>;
std::mutex g_tune_mu;
std::map<TuneKey, hg_build_opts> g_tuned;  // guarded by g_tune_mu

// Average time of `reps` builds with options o into t (after one warm-up),
// timed with events on the stream.
hg_status time_builds(hg_table* t, const void* keys, uint64_t n, uint64_t V, uint64_t seed,
                      const hg_build_opts& o, int reps, hipStream_t s, double* ms) {
    HG_CALL_ST(build_into(t, keys, n, V, seed, &o, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    hg_status st = HG_OK;
    for (int r = 0; r < reps && e == hipSuccess && st == HG_OK; ++r)
        st = build_into(t, keys, n, V, seed, &o, s);
    if (e == hipSuccess && st == HG_OK) e = hipEventRecord(e1, s);
    if (e == hipSuccess && st == HG_OK) e = hipEventSynchronize(e1);
    float f = 0.f;
    if (e == hipSuccess && st == HG_OK) e = hipEventElapsedTime(&f, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != HG_OK) return st;
    if (e != hipSuccess) return from_hip(e);
    *ms = (double)f / reps;
    return HG_OK;
}

}  // namespace

extern "C" {

const char* hg_status_string(hg_status s) {
    switch (s) {
        case HG_OK: return "ok";
        case HG_ERR_INVALID_ARG: return "invalid argument";
        case HG_ERR_OOM: return "out of device memory";
        case HG_ERR_DEVICE: return "HIP runtime error or no usable device";
        case HG_ERR_CAPACITY: return "output capacity too small";
        case HG_ERR_MISMATCH: return "tables differ in key width, hash range or seed";
        case HG_ERR_BUDGET: return "request exceeds the memory budget";
        case HG_ERR_NOT_FOUND: return "unknown table or request";
        case HG_ERR_TOO_LARGE: return "size exceeds the fixed limit of this entry point";
    }
    return "unknown status";
}

uint32_t hg_version(void) { return 100; }

hg_status hg_set_allocator(hg_alloc_fn alloc_fn, hg_free_fn free_fn, void* ctx) {
    if (!alloc_fn != !free_fn) return HG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_hook_mu);
    g_hook.alloc = alloc_fn;
    g_hook.free = free_fn;
    g_hook.ctx = alloc_fn ? ctx : nullptr;
    return HG_OK;
}

hg_status hg_hash(const void* d_keys, uint64_t n, int key_bits, uint64_t hash_range,
                  uint64_t seed, uint32_t* d_buckets, hipStream_t stream) {
    if (!valid_kb(key_bits) || !valid_range(hash_range) || n > kU32Max) return HG_ERR_INVALID_ARG;
    if (n && (!d_keys || !d_buckets)) return HG_ERR_INVALID_ARG;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    hipError_t e = key_bits == 32
                       ? run_hash<uint32_t>((const uint32_t*)d_keys, n, hash_range, seed, d_buckets, stream)
                       : run_hash<uint64_t>((const uint64_t*)d_keys, n, hash_range, seed, d_buckets, stream);
    return from_hip(e);
}

hg_status hg_histogram(const void* d_keys, uint64_t n, int key_bits, uint64_t hash_range,
                       uint64_t seed, uint32_t* d_counts, hipStream_t stream) {
    if (!valid_kb(key_bits) || !valid_range(hash_range) || n > kU32Max) return HG_ERR_INVALID_ARG;
    if ((n && !d_keys) || !d_counts) return HG_ERR_INVALID_ARG;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    hipError_t e = key_bits == 32
                       ? run_histogram<uint32_t>((const uint32_t*)d_keys, n, hash_range, seed, d_counts, 0, false, stream)
                       : run_histogram<uint64_t>((const uint64_t*)d_keys, n, hash_range, seed, d_counts, 0, false, stream);
    return from_hip(e);
}

hg_status hg_exclusive_scan(const uint32_t* d_counts, uint64_t V, uint32_t* d_offsets,
                            hipStream_t stream) {
    if (V > kU32Max || !d_offsets || (V && !d_counts)) return HG_ERR_INVALID_ARG;
    if (V && d_counts == d_offsets) return HG_ERR_INVALID_ARG;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    Workspace ws(stream);
    HG_CALL(ws.get(scan_ws_bytes(V)));
    return from_hip(scan_excl<uint32_t>(d_counts, V, d_offsets, nullptr, ws.p, stream));
}

hg_status hg_build_plan(uint64_t n, uint64_t hash_range, int key_bits, uint32_t bins,
                        hg_plan_info* out) {
    if (!out || !valid_kb(key_bits) || !valid_range(hash_range) || n > kU32Max ||
        (bins && bins > hash_range))
        return HG_ERR_INVALID_ARG;
    const V2Plan p = plan_v2(n, hash_range, key_bits, bins);
    *out = hg_plan_info{};
    out->bucket_bits = p.k;
    out->bins = p.bins;
    out->passes = p.tiers;
    out->digit_bits[0] = p.b1;
    out->digit_bits[1] = p.tiers == 2 ? p.b2 : 0u;
    out->tiles[0] = p.ntiles1;
    out->tiles[1] = p.tiers == 2 ? p.ntiles2_ub : 0u;
    out->tile_keys = kPartTile;
    out->workspace_bytes = build_ws_bytes(HG_VARIANT_V2, n, hash_range, key_bits, bins);
    return HG_OK;
}

hg_status hg_build_tune(const void* d_keys, uint64_t n, int key_bits, uint64_t hash_range,
                        uint64_t seed, const hg_build_opts* base, hipStream_t stream,
                        hg_build_opts* out, hg_tune_info* info) {
    if (!out || !valid_kb(key_bits) || !valid_range(hash_range) || n > kU32Max || (n && !d_keys))
        return HG_ERR_INVALID_ARG;
    hg_build_opts o = base ? *base : hg_build_opts{};
    if (o.variant == HG_VARIANT_AUTO) o.variant = HG_VARIANT_V2;
    if ((o.variant != HG_VARIANT_V1 && o.variant != HG_VARIANT_V2) ||
        (o.stable && (o.variant == HG_VARIANT_V1 || o.any_order)) ||
        (o.bins && o.bins > hash_range) || (o.block && (o.block % 64 || o.block > 1024)))
        return HG_ERR_INVALID_ARG;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    const bool v1 = o.variant == HG_VARIANT_V1;
    // the launch parameters are the tuner's to choose
    o.bins = 0;
    o.block = 0;
    o.v1_plain = 0;
    hg_table* t = nullptr;
    HG_CALL_ST(alloc_table(n, hash_range, key_bits, true, &t));
    struct Guard {
        hg_table* t;
        ~Guard() { hg_table_free(t); }
    } guard{t};
    double def_ms = 0.0;
    HG_CALL_ST(time_builds(t, d_keys, n, hash_range, seed, o, 2, stream, &def_ms));
    // skew class of these keys, from the table just built
    Workspace ws(stream);
    HG_CALL(ws.get(256));
    HG_CALL(max_bucket_len(t->offsets, hash_range, (uint32_t*)ws.p, stream));
    uint32_t max_len = 0;
    HG_CALL(hipMemcpyAsync(&max_len, ws.p, 4, hipMemcpyDeviceToHost, stream));
    HG_CALL(hipStreamSynchronize(stream));
    const uint32_t skew = skew_class_of(max_len, key_bits);
    const TuneKey key{log2_ceil(n ? n : 1), log2_ceil(hash_range), key_bits, o.variant,
                      o.any_order ? 1 : 0, o.stable ? 1 : 0, o.no_index ? 1 : 0, skew};
    hg_tune_info ti{};
    ti.default_ms = def_ms;
    ti.skew_class = skew;
    ti.max_bucket = max_len;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            *out = it->second;
            ti.cached = 1;
        }
    }
    if (ti.cached) {
        HG_CALL_ST(time_builds(t, d_keys, n, hash_range, seed, *out, 2, stream, &ti.ms));
        if (info) *info = ti;
        return HG_OK;
    }
    // candidates: V1 -- threads per block and merged / per-key atomics;
    // V2 -- the bin size (keys per final bin 1024, 2048, 4096 for 32-bit
    // keys), which sets the partition width and the per-bin LDS footprint
    std::vector<hg_build_opts> cands;
    if (v1) {
        for (uint32_t blk : {256u, 512u, 1024u})
            for (int plain : {0, 1}) {
                hg_build_opts c = o;
                c.block = blk;
                c.v1_plain = plain;
                cands.push_back(c);
            }
    } else {
        std::vector<uint32_t> seen_k;
        const uint32_t kv = log2_ceil(hash_range);
        for (double target : {1024.0, 2048.0, 4096.0}) {
            if (key_bits == 64 && target > 2048.0) continue;
            const double r = n ? target * (double)hash_range / (double)n : 1e30;
            uint32_t k = 0;
            while (k < kMaxLocalBits && (double)(1ull << (k + 1)) <= r) ++k;
            if (k > kv) k = kv;
            bool dup = false;
            for (uint32_t x : seen_k) dup |= x == k;
            if (dup) continue;
            seen_k.push_back(k);
            hg_build_opts c = o;
            c.bins = (uint32_t)ceil_div(hash_range, 1ull << k);
            cands.push_back(c);
        }
    }
    hg_build_opts best = o;
    double best_ms = def_ms;
    for (const hg_build_opts& c : cands) {
        double ms = 0.0;
        HG_CALL_ST(time_builds(t, d_keys, n, hash_range, seed, c, 2, stream, &ms));
        ++ti.candidates;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[key] = best;
    }
    *out = best;
    ti.ms = best_ms;
    if (info) *info = ti;
    return HG_OK;
}

hg_status hg_table_create(uint64_t n_capacity, uint64_t range_capacity, int key_bits,
                          hg_table** out) {
    if (!out || !valid_kb(key_bits) || !valid_range(range_capacity) || n_capacity > kU32Max)
        return HG_ERR_INVALID_ARG;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    return alloc_table(n_capacity, range_capacity, key_bits, true, out);
}

hg_status hg_table_build(hg_table* t, const void* d_keys, uint64_t n, uint64_t hash_range,
                         uint64_t seed, const hg_build_opts* opts, hipStream_t stream) {
    if (!t || !valid_range(hash_range) || n > kU32Max || (n && !d_keys)) return HG_ERR_INVALID_ARG;
    if (n > t->n_cap || hash_range > t->V_cap) return HG_ERR_CAPACITY;
    return build_into(t, d_keys, n, hash_range, seed, opts, stream);
}

hg_status hg_build(const void* d_keys, uint64_t n, int key_bits, uint64_t hash_range,
                   uint64_t seed, const hg_build_opts* opts, hipStream_t stream, hg_table** out) {
    if (!out || !valid_kb(key_bits) || !valid_range(hash_range) || n > kU32Max ||
        (n && !d_keys))
        return HG_ERR_INVALID_ARG;
    if (opts && ((opts->variant != 0 && opts->variant != 1 && opts->variant != 2) ||
                 (opts->stable && opts->variant == HG_VARIANT_V1) ||
                 (opts->bins && opts->bins > hash_range)))
        return HG_ERR_INVALID_ARG;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    hg_table* t = nullptr;
    hg_status st = alloc_table(n, hash_range, key_bits, false, &t);
    if (st != HG_OK) return st;
    st = build_into(t, d_keys, n, hash_range, seed, opts, stream);
    if (st != HG_OK) {
        hg_table_free(t);
        return st;
    }
    *out = t;
    return HG_OK;
}

hg_status hg_table_view(const hg_table* t, hg_table_info* info) {
    if (!t || !info) return HG_ERR_INVALID_ARG;
    info->d_offsets = t->offsets;
    info->d_ids = t->ids;
    info->d_keys = t->keys;
    info->n = t->n;
    info->hash_range = t->V;
    info->seed = t->seed;
    info->key_bits = t->key_bits;
    info->variant = t->variant;
    info->device_bytes = t->bytes;
    return HG_OK;
}

hg_status hg_table_export(const hg_table* t, uint32_t* d_offsets, uint32_t* d_ids, void* d_keys,
                          hipStream_t stream) {
    if (!t || t->V == 0) return HG_ERR_INVALID_ARG;
    if (t->has_len) {
        // compacted CSR of the live entries
        Workspace ws(stream);
        HG_CALL(ws.get(align_up((t->V + 1) * 4, 256) + scan_ws_bytes(t->V)));
        Carver c(ws.p);
        uint32_t* own = c.take<uint32_t>(t->V + 1);
        uint32_t* off = d_offsets ? d_offsets : own;
        void* sws = c.take<char>(scan_ws_bytes(t->V));
        HG_CALL(scan_excl<uint32_t>(t->len, t->V, off, nullptr, sws, stream));
        const TableDev d = dev_view(t);
        HG_CALL(t->key_bits == 32
                    ? run_export_live<uint32_t>(d, t->len, off, d_ids, (uint32_t*)d_keys, stream)
                    : run_export_live<uint64_t>(d, t->len, off, d_ids, (uint64_t*)d_keys, stream));
        return HG_OK;
    }
    if (d_offsets)
        HG_CALL(hipMemcpyAsync(d_offsets, t->offsets, (t->V + 1) * 4, hipMemcpyDeviceToDevice, stream));
    if (d_ids && t->n)
        HG_CALL(hipMemcpyAsync(d_ids, t->ids, t->n * 4, hipMemcpyDeviceToDevice, stream));
    if (d_keys && t->n)
        HG_CALL(hipMemcpyAsync(d_keys, t->keys, t->n * key_size(t->key_bits),
                               hipMemcpyDeviceToDevice, stream));
    return HG_OK;
}

hg_status hg_table_erase(hg_table* t, const void* d_keys, uint64_t m, uint64_t* h_removed,
                         hipStream_t stream) {
    if (!t || t->V == 0 || (m && !d_keys)) return HG_ERR_INVALID_ARG;
    if (!t->has_head) return HG_ERR_INVALID_ARG;  // needs a V2 table with the probe index
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    if (!t->len) {
        HG_CALL(hipMalloc((void**)&t->len, t->V_cap * 4));
        HG_CALL(hipMalloc((void**)&t->dead, t->n_cap ? t->n_cap : 1));
        HG_CALL(hipMalloc((void**)&t->touched, t->V_cap));
        t->bytes += t->V_cap * 5 + (t->n_cap ? t->n_cap : 1);
        HG_CALL(hipMemsetAsync(t->dead, 0, t->n_cap ? t->n_cap : 1, stream));
        HG_CALL(hipMemsetAsync(t->touched, 0, t->V_cap, stream));
    }
    if (!t->has_len) {
        HG_CALL(init_lengths(t->offsets, t->V, t->len, stream));
        t->has_len = true;
    }
    Workspace ws(stream);
    HG_CALL(ws.get(256));
    unsigned long long* d_removed = (unsigned long long*)ws.p;
    HG_CALL(fill_u32((uint32_t*)d_removed, 2, 0u, stream));
    const TableDev d = dev_view(t);
    HG_CALL(t->key_bits == 32
                ? run_erase<uint32_t>(d, t->len, t->dead, t->touched, t->head,
                                      (const uint32_t*)d_keys, m, d_removed, stream)
                : run_erase<uint64_t>(d, t->len, t->dead, t->touched, t->head,
                                      (const uint64_t*)d_keys, m, d_removed, stream));
    uint64_t removed = 0;
    const hg_status st = read_u64((const uint64_t*)d_removed, &removed, stream);
    if (st != HG_OK) return st;
    t->live -= removed;
    if (h_removed) *h_removed = removed;
    return HG_OK;
}

hg_status hg_table_lengths(const hg_table* t, const uint32_t** d_lengths, uint64_t* live) {
    if (!t || (!d_lengths && !live)) return HG_ERR_INVALID_ARG;
    if (d_lengths) *d_lengths = t->has_len ? t->len : nullptr;
    if (live) *live = t->live;
    return HG_OK;
}

struct hg_collection {
    int key_bits = 32;
    uint64_t seed = 0;
    int32_t shift = 0;
    uint32_t S = 0;
    uint64_t n = 0, buckets = 0, heavy_keys = 0, bytes = 0;
    uint32_t* set_off = nullptr;
    uint64_t* bb = nullptr;
    uint32_t* offsets = nullptr;
    uint32_t* ids = nullptr;
    void* keys = nullptr;
};

namespace {

void coll_release(hg_collection* c) {
    if (c->set_off) (void)hipFree(c->set_off);
    if (c->bb) (void)hipFree(c->bb);
    if (c->offsets) (void)hipFree(c->offsets);
    if (c->ids) (void)hipFree(c->ids);
    if (c->keys) (void)hipFree(c->keys);
    delete c;
}

hg_status coll_build_into(hg_collection* c, const void* d_keys, const uint32_t* d_set_offsets,
                          hipStream_t stream) {
    const uint32_t S = c->S;
    HG_CALL(hipMalloc((void**)&c->set_off, ((uint64_t)S + 1) * 4));
    HG_CALL(hipMalloc((void**)&c->bb, ((uint64_t)S + 2) * 8));
    HG_CALL(hipMemcpyAsync(c->set_off, d_set_offsets, ((uint64_t)S + 1) * 4,
                           hipMemcpyDeviceToDevice, stream));
    Workspace pws(stream);
    HG_CALL(pws.get(coll_plan_ws_bytes(S)));
    CollPlan plan{};
    HG_CALL(coll_plan(c->set_off, S, c->shift, pws.p, c->bb, &plan, stream));
    if (plan.bad || plan.buckets >= kU32Max || (plan.n && !d_keys)) return HG_ERR_INVALID_ARG;
    c->n = plan.n;
    c->buckets = plan.buckets;
    c->heavy_keys = plan.big_keys;
    const size_t ks = key_size(c->key_bits);
    HG_CALL(hipMalloc((void**)&c->offsets, (plan.buckets + 1) * 4));
    HG_CALL(hipMalloc((void**)&c->ids, (plan.n ? plan.n : 1) * 4));
    HG_CALL(hipMalloc(&c->keys, (plan.n ? plan.n : 1) * ks));
    c->bytes = ((uint64_t)S + 1) * 4 + ((uint64_t)S + 2) * 8 + (plan.buckets + 1) * 4 +
               plan.n * (4 + ks);
    Workspace bws(stream);
    HG_CALL(bws.get(coll_build_ws_bytes(plan, c->key_bits)));
    bool bad = false;
    HG_CALL(c->key_bits == 32
                ? run_coll_build<uint32_t>((const uint32_t*)d_keys, c->set_off, S, c->seed, c->bb,
                                           plan, bws.p, c->offsets, c->ids, (uint32_t*)c->keys,
                                           &bad, stream)
                : run_coll_build<uint64_t>((const uint64_t*)d_keys, c->set_off, S, c->seed, c->bb,
                                           plan, bws.p, c->offsets, c->ids, (uint64_t*)c->keys,
                                           &bad, stream));
    return bad ? HG_ERR_DEVICE : HG_OK;
}

CollDev coll_view(const hg_collection* c) {
    return CollDev{c->set_off, c->bb, c->offsets, c->ids, c->keys, c->S};
}

}  // namespace

hg_status hg_collection_build(const void* d_keys, const uint32_t* d_set_offsets, uint32_t sets,
                              int key_bits, uint64_t seed, int32_t range_shift,
                              hg_collection** out, hipStream_t stream) {
    if (!out) return HG_ERR_INVALID_ARG;
    *out = nullptr;
    if (!d_set_offsets || !valid_kb(key_bits) || range_shift < -31 || range_shift > 31 ||
        sets >= 0xfffffffeu)
        return HG_ERR_INVALID_ARG;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    hg_collection* c = new (std::nothrow) hg_collection();
    if (!c) return HG_ERR_OOM;
    c->key_bits = key_bits;
    c->seed = seed;
    c->shift = range_shift;
    c->S = sets;
    const hg_status st = coll_build_into(c, d_keys, d_set_offsets, stream);
    if (st != HG_OK) {
        (void)hipStreamSynchronize(stream);
        coll_release(c);
        return st;
    }
    *out = c;
    return HG_OK;
}

hg_status hg_collection_view(const hg_collection* c, hg_collection_info* info) {
    if (!c || !info) return HG_ERR_INVALID_ARG;
    *info = hg_collection_info{};
    info->sets = c->S;
    info->key_bits = c->key_bits;
    info->seed = c->seed;
    info->range_shift = c->shift;
    info->n = c->n;
    info->buckets = c->buckets;
    info->heavy_keys = c->heavy_keys;
    info->bytes = c->bytes;
    info->d_set_offsets = c->set_off;
    info->d_bucket_base = c->bb;
    info->d_offsets = c->offsets;
    info->d_ids = c->ids;
    info->d_keys = c->keys;
    return HG_OK;
}

hg_status hg_collection_export(const hg_collection* c, uint64_t* d_bucket_base,
                               uint32_t* d_offsets, uint32_t* d_ids, void* d_keys,
                               hipStream_t stream) {
    if (!c) return HG_ERR_INVALID_ARG;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    if (d_bucket_base)
        HG_CALL(hipMemcpyAsync(d_bucket_base, c->bb, ((uint64_t)c->S + 2) * 8, k, stream));
    if (d_offsets) HG_CALL(hipMemcpyAsync(d_offsets, c->offsets, (c->buckets + 1) * 4, k, stream));
    if (d_ids && c->n) HG_CALL(hipMemcpyAsync(d_ids, c->ids, c->n * 4, k, stream));
    if (d_keys && c->n)
        HG_CALL(hipMemcpyAsync(d_keys, c->keys, c->n * key_size(c->key_bits), k, stream));
    return HG_OK;
}

hg_status hg_collection_intersect(const hg_collection* a, const hg_collection* b,
                                  const uint32_t* d_pairs, uint64_t pairs, uint64_t* d_counts,
                                  uint64_t* h_total, hipStream_t stream) {
    if (!a || !b || (pairs && !d_pairs) || (!d_counts && !h_total)) return HG_ERR_INVALID_ARG;
    if (a->key_bits != b->key_bits || a->seed != b->seed) return HG_ERR_MISMATCH;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    if (h_total) *h_total = 0;
    Workspace ws(stream);
    HG_CALL(ws.get(coll_pairs_ws_bytes(pairs)));
    bool bad = false;
    HG_CALL(a->key_bits == 32
                ? run_coll_intersect<uint32_t>(coll_view(a), coll_view(b), a->seed, d_pairs, pairs,
                                               (unsigned long long*)d_counts, h_total, ws.p, &bad,
                                               stream)
                : run_coll_intersect<uint64_t>(coll_view(a), coll_view(b), a->seed, d_pairs, pairs,
                                               (unsigned long long*)d_counts, h_total, ws.p, &bad,
                                               stream));
    return bad ? HG_ERR_INVALID_ARG : HG_OK;
}

void hg_collection_free(hg_collection* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    coll_release(c);
}

void hg_table_free(hg_table* t) {
    if (!t) return;
    if (t->offsets) (void)hipFree(t->offsets);
    if (t->ids) (void)hipFree(t->ids);
    if (t->keys) (void)hipFree(t->keys);
    if (t->head) (void)hipFree(t->head);
    if (t->len) (void)hipFree(t->len);
    if (t->dead) (void)hipFree(t->dead);
    if (t->touched) (void)hipFree(t->touched);
    if (t->runs.kperm) (void)hipFree(t->runs.kperm);
    if (t->runs.run_key) (void)hipFree(t->runs.run_key);
    if (t->runs.run_end) (void)hipFree(t->runs.run_end);
    if (t->ws) (void)hipFree(t->ws);
    delete t;
}

hg_status hg_probe_ordered(const hg_table* t, const void* d_queries, uint64_t m,
                           uint32_t* d_counts, uint64_t* h_total, int32_t order,
                           hipStream_t stream) {
    if (check_table_arg(t) != HG_OK || m > kU32Max || (m && !d_queries)) return HG_ERR_INVALID_ARG;
    if (!d_counts && !h_total) return HG_ERR_INVALID_ARG;
    if (order != HG_PROBE_AUTO && order != HG_PROBE_INPUT_ORDER && order != HG_PROBE_GROUPED &&
        order != HG_PROBE_GROUPED_UNLESS_SKEWED)
        return HG_ERR_INVALID_ARG;
    if (t->V == 0) return HG_ERR_INVALID_ARG;  // never built
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    TableDev d = dev_view(t);
    bool grouped = order == HG_PROBE_GROUPED || order == HG_PROBE_GROUPED_UNLESS_SKEWED;
    if (order == HG_PROBE_AUTO)  // where grouping measured faster on MI355X
        grouped = d.head != nullptr && m >= t->V / 2 &&
                  t->V >= (d_counts ? (1ull << 27) : (1ull << 26));
    grouped = grouped && m > 0;
    const size_t kbytes = t->key_bits / 8;
    const size_t tot_bytes = h_total ? align_up(probe_total_slots(m) * 8, 256) : 0;
    Workspace ws(stream);
    hipError_t ae =
        ws.get(tot_bytes + (grouped ? probe_grouped_ws_bytes(m, t->V, kbytes) : 0) + 256);
    if (ae == hipErrorOutOfMemory && grouped && order == HG_PROBE_AUTO) {
        // the grouping's workspace is out of reach: probe in input order
        (void)hipGetLastError();  // the failed allocation's error is not the probe's
        ws.p = nullptr;
        grouped = false;
        ae = ws.get(tot_bytes + 256);
    }
    if (ae != hipSuccess) return from_hip(ae);
    unsigned long long* d_total = h_total ? (unsigned long long*)ws.p : nullptr;
    void* gws = (char*)ws.p + tot_bytes;
    hipError_t e;
    // skewed queries keep input order, decided on the device
    const bool decide = order == HG_PROBE_AUTO || order == HG_PROBE_GROUPED_UNLESS_SKEWED;
    if (grouped)
        e = t->key_bits == 32
                ? run_probe_grouped<uint32_t>(d, (const uint32_t*)d_queries, m, d_counts, d_total, gws, stream, decide)
                : run_probe_grouped<uint64_t>(d, (const uint64_t*)d_queries, m, d_counts, d_total, gws, stream, decide);
    else
        e = t->key_bits == 32
                ? run_probe_counts<uint32_t>(d, (const uint32_t*)d_queries, m, d_counts, d_total, stream)
                : run_probe_counts<uint64_t>(d, (const uint64_t*)d_queries, m, d_counts, d_total, stream);
    if (e != hipSuccess) return from_hip(e);
    if (h_total) return read_u64((const uint64_t*)d_total, h_total, stream);
    return HG_OK;
}

hg_status hg_probe(const hg_table* t, const void* d_queries, uint64_t m, uint32_t* d_counts,
                   uint64_t* h_total, hipStream_t stream) {
    return hg_probe_ordered(t, d_queries, m, d_counts, h_total, HG_PROBE_AUTO, stream);
}

hg_status hg_probe_pairs(const hg_table* t, const void* d_queries, uint64_t m,
                         uint32_t* d_build_ids, uint32_t* d_probe_ids, uint64_t capacity,
                         uint64_t* h_total, hipStream_t stream) {
    HG_CALL_ST(check_pairs_args(t, d_queries, m, d_build_ids, d_probe_ids, capacity, h_total));
    if (m == 0) {
        *h_total = 0;
        return HG_OK;
    }
    Workspace ws(stream);
    HG_CALL(ws.get(probe_ws_bytes(m) + align_up(m, 256)));
    return probe_pairs_into(t, d_queries, m, d_build_ids, d_probe_ids, capacity, h_total, ws.p,
                            stream, true);
}

hg_status hg_probe_pairs_noalloc(const hg_table* t, const void* d_queries, uint64_t m,
                                 uint32_t* d_build_ids, uint32_t* d_probe_ids, uint64_t capacity,
                                 uint64_t* h_total, hipStream_t stream) {
    HG_CALL_ST(check_pairs_args(t, d_queries, m, d_build_ids, d_probe_ids, capacity, h_total));
    if (m > HG_NOALLOC_MAX_QUERIES) return HG_ERR_TOO_LARGE;
    if (m == 0) {
        *h_total = 0;
        return HG_OK;
    }
    void* ws = nullptr;
    HG_CALL_ST(static_scratch(probe_ws_bytes(m), &ws));
    return probe_pairs_into(t, d_queries, m, d_build_ids, d_probe_ids, capacity, h_total, ws,
                            stream, false);
}

hg_status hg_intersect_edges(const hg_table* a, const hg_table* b, uint32_t* d_counts_edges,
                             uint64_t* h_total, hipStream_t stream) {
    if (!a || !b || (!d_counts_edges && !h_total)) return HG_ERR_INVALID_ARG;
    if (a->V == 0 || b->V == 0) return HG_ERR_INVALID_ARG;
    if (a->key_bits != b->key_bits || a->V != b->V || a->seed != b->seed) return HG_ERR_MISMATCH;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    if (b->n == 0) {
        if (h_total) *h_total = 0;
        return HG_OK;
    }
    Workspace ws(stream);
    unsigned long long* d_total = nullptr;
    if (h_total) {
        HG_CALL(ws.get(probe_total_slots(b->n) * 8));
        d_total = (unsigned long long*)ws.p;
    }
    const TableDev da = dev_view(a), db = dev_view(b);
    HG_CALL(a->key_bits == 32
                ? run_intersect_counts<uint32_t>(da, db, d_counts_edges, nullptr, d_total, stream)
                : run_intersect_counts<uint64_t>(da, db, d_counts_edges, nullptr, d_total, stream));
    if (h_total) return read_u64((const uint64_t*)d_total, h_total, stream);
    return HG_OK;
}

hg_status hg_intersect(const hg_table* a, const hg_table* b, uint32_t* d_counts_b,
                       uint32_t* d_a_ids, uint32_t* d_b_ids, uint64_t capacity,
                       uint64_t* h_total, hipStream_t stream) {
    if (!a || !b) return HG_ERR_INVALID_ARG;
    if (capacity && (!d_a_ids || !d_b_ids || !h_total)) return HG_ERR_INVALID_ARG;
    if (!d_counts_b && !h_total) return HG_ERR_INVALID_ARG;
    if (a->V == 0 || b->V == 0) return HG_ERR_INVALID_ARG;
    if (a->key_bits != b->key_bits || a->V != b->V || a->seed != b->seed) return HG_ERR_MISMATCH;
    if (device_ready() != HG_OK) return HG_ERR_DEVICE;
    const uint64_t nb = b->n;
    if (nb == 0) {
        if (h_total) *h_total = 0;
        return HG_OK;
    }
    TableDev da = dev_view(a), db = dev_view(b);
    const bool pairs = capacity > 0;
    // Counts by B's input index: Alg. 3 writes them in B's edge order, then
    // they are scattered through B's ids (a permutation of B's inputs) in
    // L2-sized windows.  After an erase B's ids hold stale copies, so the
    // counts are scattered one by one as they are found instead.
    const bool staged = d_counts_b && !b->has_len;
    Workspace ws(stream);
    HG_CALL(ws.get(probe_ws_bytes(nb) + probe_total_slots(nb) * 8 + 512 +
                   (staged ? scatter_perm_ws_bytes(nb) : 0)));
    Carver c(ws.p);
    uint32_t* edge = c.take<uint32_t>(nb);
    uint64_t* pos = c.take<uint64_t>(nb + 1);
    void* scan_ws = c.take<char>(scan_ws_bytes(nb));
    unsigned long long* d_total = (unsigned long long*)c.take<uint64_t>(probe_total_slots(nb));
    void* sc_ws = staged ? c.take<char>(scatter_perm_ws_bytes(nb)) : nullptr;
    uint32_t* by_edge = (pairs || staged) ? edge : nullptr;
    uint32_t* by_input = staged ? nullptr : d_counts_b;
    hipError_t e = a->key_bits == 32
                       ? run_intersect_counts<uint32_t>(da, db, by_edge, by_input,
                                                        (h_total && !pairs) ? d_total : nullptr, stream)
                       : run_intersect_counts<uint64_t>(da, db, by_edge, by_input,
                                                        (h_total && !pairs) ? d_total : nullptr, stream);
    if (e != hipSuccess) return from_hip(e);
    if (staged) HG_CALL(scatter_perm(db.ids, edge, nb, d_counts_b, sc_ws, stream));
    if (!pairs) {
        if (h_total) return read_u64((const uint64_t*)d_total, h_total, stream);
        return HG_OK;
    }
    HG_CALL(scan_excl<uint64_t>(edge, nb, pos, nullptr, scan_ws, stream));
    hg_status st = read_u64(pos + nb, h_total, stream);
    if (st != HG_OK) return st;
    if (*h_total > capacity) return HG_ERR_CAPACITY;
    if (*h_total == 0) return HG_OK;
    e = a->key_bits == 32 ? run_intersect_pairs<uint32_t>(da, db, pos, d_a_ids, d_b_ids, stream)
                          : run_intersect_pairs<uint64_t>(da, db, pos, d_a_ids, d_b_ids, stream);
    if (e != hipSuccess) return from_hip(e);
    HG_CALL(hipStreamSynchronize(stream));
    return HG_OK;
}

}  // extern "C"
