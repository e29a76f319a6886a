// Batched HashGraph build + probe: many independent tables of uneven size in
// one hipGraph launch.
//
// Every table is built exactly as hg_build's V2 path builds it (same stable
// layout) and probed as hg_probe does; what changes is the launch structure.
// The work items of all tables -- partition tiles, final bins and probe
// tiles -- are numbered in one global index space per kernel, with per-table
// descriptors on the device and prefix arrays that a workgroup searches to
// find its table.  Tables small enough to be a single bin that fits in LDS
// (n <= 3072 here) skip the partition entirely: their bin is built straight
// from the caller's keys.  Larger tables take one stable partition pass into
// a shared workspace, then the per-bin LDS build.  The six kernels of a run
// (clear, tile histograms, per-table column scan, partition, per-bin build,
// oversize bins, probe) are captured once into a hipGraph; a run is a single
// graph launch.  The bin-size target (keys per final bin, which sets the
// partition fan-out and the LDS footprint) is chosen by timing candidate
// graphs on the actual batch.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "hashgraph.h"
#include "hg_v2_device.h"

namespace hg {

namespace {

using namespace v2dev;

// Launch shapes the tuner chooses between (defaults first): keys per thread
// of the partition tiles (256 threads each), and threads x queries per thread
// of the probe workgroups.
constexpr uint32_t kPartItemsChoices[] = {16u, 8u};
struct ProbeShape {
    uint32_t threads, items;
};
constexpr ProbeShape kProbeShapes[] = {{256u, 4u}, {256u, 8u}, {512u, 2u}, {128u, 8u}};

enum : uint32_t { kDirect = 0, kPartitioned = 1, kEmpty = 2 };

template <typename Key>
struct BTable {
    const Key* keys;
    const Key* queries;
    uint32_t* offsets;
    uint32_t* ids;
    Key* ekeys;
    uint32_t* counts;
    typename KeyTraits<Key>::Params hp;
    uint32_t n, m, V;
    uint32_t kind;      // kDirect / kPartitioned / kEmpty
    uint32_t k;         // log2 buckets per bin
    uint32_t b1;        // partition digit bits (kPartitioned)
    uint32_t bins;      // final bins
    uint32_t ntiles;    // partition tiles (kPartitioned)
    uint32_t mat_base;  // first matrix entry
    uint32_t key_base;  // first slot in the shared partition workspace
};

struct BPrefix {
    const uint32_t* tile;   // [T+1] first partition tile of each table
    const uint32_t* bin;    // [T+1] first final bin
    const uint32_t* qtile;  // [T+1] first probe tile
    uint32_t T;
};

__device__ __forceinline__ uint32_t find_table(const uint32_t* __restrict__ pre, uint32_t T,
                                               uint32_t x) {
    uint32_t lo = 0, hi = T;  // largest i with pre[i] <= x
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_bclear(uint32_t* heavy_count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *heavy_count = 0;
}

template <typename Key, int IT>
__global__ __launch_bounds__(kPartThreads) void k_bhist(const BTable<Key>* __restrict__ tabs,
                                                        BPrefix pre, uint32_t tiles,
                                                        uint32_t* __restrict__ mat) {
    constexpr uint32_t TILE = kPartThreads * IT;
    extern __shared__ uint32_t cnt[];
    const uint32_t t = xcd_tile(blockIdx.x, tiles);
    if (t >= tiles) return;
    const uint32_t i = find_table(pre.tile, pre.T, t);
    const BTable<Key>& tb = tabs[i];
    const uint32_t lt = t - pre.tile[i];
    const uint32_t D = 1u << tb.b1;
    const uint32_t begin = lt * TILE;
    const uint32_t end = (tb.n - begin > TILE) ? begin + TILE : tb.n;
    for (uint32_t d = threadIdx.x; d < D; d += kPartThreads) cnt[d] = 0;
    Key k[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t x = begin + r * kPartThreads + threadIdx.x;
        k[r] = (x < end) ? tb.keys[x] : (Key)0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t x = begin + r * kPartThreads + threadIdx.x;
        if (x < end) atomicAdd(&cnt[(KeyTraits<Key>::bucket(k[r], tb.hp) >> tb.k) & (D - 1)], 1u);
    }
    __syncthreads();
    uint32_t* row = mat + tb.mat_base + (size_t)lt * D;
    for (uint32_t d = threadIdx.x; d < D; d += kPartThreads) row[d] = cnt[d];
}

// One workgroup per table: turn its [tile][digit] counts into absolute bases
// key_base + (keys of smaller digits) + (keys of this digit in earlier tiles).
template <typename Key>
__global__ __launch_bounds__(256) void k_bcolscan(const BTable<Key>* __restrict__ tabs,
                                                  uint32_t* __restrict__ mat) {
    __shared__ uint32_t tmp[256 / kWave + 1];
    const BTable<Key>& tb = tabs[blockIdx.x];
    if (tb.kind != kPartitioned) return;
    const uint32_t D = 1u << tb.b1, nt = tb.ntiles;
    uint32_t* m = mat + tb.mat_base;
    const uint32_t per = (D + 255) / 256;  // <= 8
    const uint32_t d0 = threadIdx.x * per;
    uint32_t tot[8];
    uint32_t mine = 0;
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t d = d0 + j;
        uint32_t acc = 0;
        if (d < D)
            for (uint32_t t = 0; t < nt; ++t) acc += m[(size_t)t * D + d];
        tot[j] = acc;
        mine += acc;
    }
    uint32_t all;
    uint32_t run = tb.key_base + block_excl_scan<256>(mine, tmp, &all);
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t d = d0 + j;
        if (d < D) {
            uint32_t r = run;
            for (uint32_t t = 0; t < nt; ++t) {
                const uint32_t v = m[(size_t)t * D + d];
                m[(size_t)t * D + d] = r;
                r += v;
            }
        }
        run += tot[j];
    }
}

// STABLE: equal digits keep their order; otherwise their order is
// unspecified (ranked with LDS atomics, no ballots).
template <typename Key, bool STABLE, int IT>
__global__ __launch_bounds__(kPartThreads) void k_bpart(const BTable<Key>* __restrict__ tabs,
                                                        BPrefix pre, uint32_t tiles,
                                                        const uint32_t* __restrict__ mat,
                                                        Key* __restrict__ rkeys,
                                                        uint32_t* __restrict__ rids) {
    constexpr uint32_t TILE = kPartThreads * IT;
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t t = xcd_tile(blockIdx.x, tiles);
    if (t >= tiles) return;
    const uint32_t i = find_table(pre.tile, pre.T, t);
    const BTable<Key>& tb = tabs[i];
    const uint32_t lt = t - pre.tile[i];
    const uint32_t bits = tb.b1, D = 1u << bits;
    Key* skeys = (Key*)smem;
    uint32_t* sids = (uint32_t*)(skeys + TILE);
    uint16_t* sdig = (uint16_t*)(sids + TILE);
    uint32_t* wcnt = (uint32_t*)(sdig + TILE);
    uint32_t* dstart = wcnt + W_PART * D;
    uint32_t* tbase = dstart + D;
    uint32_t* tmp = tbase + D;
    const uint32_t begin = lt * TILE;
    const uint32_t cnt = (tb.n - begin > TILE) ? TILE : tb.n - begin;
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t wbase = w * (kWave * IT);
    Key k[IT];
    uint32_t dig[IT], pos[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t e = wbase + r * kWave + lane;
        k[r] = (e < cnt) ? tb.keys[begin + e] : (Key)0;
    }
    // the tile's digit bases, loaded now so that their latency overlaps the
    // ranking (D <= 2048: at most kRowPer per thread)
    constexpr int kRowPer = (1 << kMaxDigitBits) / kPartThreads;
    const uint32_t* row = mat + tb.mat_base + (size_t)lt * D;
    uint32_t rowv[kRowPer];
#pragma unroll
    for (int j = 0; j < kRowPer; ++j) {
        const uint32_t d = threadIdx.x + j * kPartThreads;
        rowv[j] = d < D ? row[d] : 0u;
    }
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t e = wbase + r * kWave + lane;
        dig[r] = (e < cnt) ? ((KeyTraits<Key>::bucket(k[r], tb.hp) >> tb.k) & (D - 1)) : D;
    }
    if (STABLE) rank_stable<kPartThreads, IT>(dig, bits, wcnt, dstart, tmp, pos);
    else rank_any<kPartThreads, IT>(dig, bits, wcnt, dstart, tmp, pos);
#pragma unroll
    for (int j = 0; j < kRowPer; ++j) {
        const uint32_t d = threadIdx.x + j * kPartThreads;
        if (d < D) tbase[d] = rowv[j] - dstart[d];
    }
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        if (dig[r] < D) {
            const uint32_t e = wbase + r * kWave + lane;
            skeys[pos[r]] = k[r];
            sids[pos[r]] = begin + e;
            sdig[pos[r]] = (uint16_t)dig[r];
        }
    }
    __syncthreads();
    const uint32_t lo = tb.key_base, len = tb.n;
    for (uint32_t p = threadIdx.x; p < cnt; p += kPartThreads) {
        const uint32_t o = tbase[sdig[p]] + p;
        if (o - lo < len) {
            rkeys[o] = skeys[p];
            rids[o] = sids[p];
        }
    }
}

// Source range of global bin gb: table, local bin and [start, end) in the
// workspace (partitioned tables) or in the table's own keys (direct tables).
template <typename Key>
__device__ __forceinline__ void bin_range(const BTable<Key>* __restrict__ tabs, const BPrefix& pre,
                                          const uint32_t* __restrict__ mat, uint32_t gb,
                                          uint32_t& i, uint32_t& lb, uint32_t& start,
                                          uint32_t& end) {
    i = find_table(pre.bin, pre.T, gb);
    const BTable<Key>& tb = tabs[i];
    lb = gb - pre.bin[i];
    if (tb.kind == kPartitioned) {
        const uint32_t* row0 = mat + tb.mat_base;
        start = row0[lb];
        end = (lb + 1 < tb.bins) ? row0[lb + 1] : tb.key_base + tb.n;
    } else {
        start = 0;
        end = tb.kind == kDirect ? tb.n : 0u;
    }
}

template <typename Key>
__global__ __launch_bounds__(kLocalThreads) void k_blocal(
    const BTable<Key>* __restrict__ tabs, BPrefix pre, uint32_t bins,
    const uint32_t* __restrict__ mat, const Key* __restrict__ rkeys,
    const uint32_t* __restrict__ rids, uint32_t* __restrict__ heavy_list,
    uint32_t* __restrict__ heavy_count, bool any_order) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t gb = blockIdx.x;
    if (gb >= bins) return;
    uint32_t i, lb, start, end;
    bin_range<Key>(tabs, pre, mat, gb, i, lb, start, end);
    const BTable<Key>& tb = tabs[i];
    const uint32_t L = end - start;
    if (lb + 1 == tb.bins && threadIdx.x == 0) tb.offsets[tb.V] = tb.n;
    if (L > light_cap<Key>()) {
        if (threadIdx.x == 0) heavy_list[atomicAdd(heavy_count, 1u)] = gb;
        return;
    }
    const uint32_t NB = 1u << tb.k, v0 = lb << tb.k;
    const uint32_t nb = (tb.V - v0 < NB) ? tb.V - v0 : NB;
    if (tb.kind == kPartitioned)
        light_bin_body<Key>(rkeys + start, rids + start, 0u, L, start - tb.key_base, v0, tb.k, nb,
                            tb.hp, tb.offsets, IndexOut{}, tb.ids, tb.ekeys, smem, any_order);
    else
        light_bin_body<Key>(tb.keys, nullptr, 0u, L, 0u, v0, tb.k, nb, tb.hp, tb.offsets, IndexOut{},
                            tb.ids, tb.ekeys, smem, any_order);
}

template <typename Key>
__global__ __launch_bounds__(kLocalThreads) void k_bheavy(
    const BTable<Key>* __restrict__ tabs, BPrefix pre, const uint32_t* __restrict__ mat,
    const Key* __restrict__ rkeys, const uint32_t* __restrict__ rids,
    const uint32_t* __restrict__ heavy_list, const uint32_t* __restrict__ heavy_count) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t nheavy = *heavy_count;
    for (uint32_t h = blockIdx.x; h < nheavy; h += gridDim.x) {
        uint32_t i, lb, start, end;
        bin_range<Key>(tabs, pre, mat, heavy_list[h], i, lb, start, end);
        const BTable<Key>& tb = tabs[i];
        const uint32_t NB = 1u << tb.k, v0 = lb << tb.k;
        const uint32_t nb = (tb.V - v0 < NB) ? tb.V - v0 : NB;
        if (tb.kind == kPartitioned)
            heavy_bin_body<Key>(rkeys + start, rids + start, 0u, end - start, start - tb.key_base,
                                v0, tb.k, nb, tb.hp, tb.offsets, IndexOut{}, tb.ids, tb.ekeys, smem);
        else
            heavy_bin_body<Key>(tb.keys, nullptr, 0u, end - start, 0u, v0, tb.k, nb, tb.hp,
                                tb.offsets, IndexOut{}, tb.ids, tb.ekeys, smem);
        __syncthreads();
    }
}

template <typename Key, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_bprobe(const BTable<Key>* __restrict__ tabs,
                                                    BPrefix pre, uint32_t qtiles) {
    // each XCD walks a contiguous range of probe tiles, so a table's
    // offsets and keys are read through one L2
    const uint32_t qt = xcd_tile(blockIdx.x, qtiles);
    if (qt >= qtiles) return;
    const uint32_t i = find_table(pre.qtile, pre.T, qt);
    const BTable<Key>& tb = tabs[i];
    const uint32_t base = (qt - pre.qtile[i]) * (THREADS * ITEMS) + threadIdx.x;
    Key q[ITEMS];
    uint32_t lo[ITEMS], hi[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t j = base + r * THREADS;
        q[r] = (j < tb.m) ? tb.queries[j] : (Key)0;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t j = base + r * THREADS;
        if (j < tb.m) {
            const uint32_t h = KeyTraits<Key>::bucket(q[r], tb.hp);
            lo[r] = tb.offsets[h];
            hi[r] = tb.offsets[h + 1];
        } else {
            lo[r] = hi[r] = 0;
        }
    }
    // the first two keys of every bucket are loaded together (one round of
    // overlapped random reads; at load 1 most buckets hold at most two keys),
    // then the rest of each bucket is scanned
    Key k0[ITEMS], k1[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        k0[r] = lo[r] < hi[r] ? tb.ekeys[lo[r]] : (Key)0;
        k1[r] = lo[r] + 1 < hi[r] ? tb.ekeys[lo[r] + 1] : (Key)0;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t j = base + r * THREADS;
        uint32_t c = (lo[r] < hi[r] && k0[r] == q[r]) ? 1u : 0u;
        c += (lo[r] + 1 < hi[r] && k1[r] == q[r]) ? 1u : 0u;
        for (uint32_t p = lo[r] + 2; p < hi[r]; ++p) c += (tb.ekeys[p] == q[r]) ? 1u : 0u;
        if (j < tb.m) tb.counts[j] = c;
    }
}

size_t part_smem_bytes(size_t key_size, uint32_t bits, uint32_t tile) {
    const size_t D = 1u << bits;
    return tile * (key_size + 4 + 2) + W_PART * D * 4 + 2 * D * 4 + (W_PART + 1) * 4 + 64;
}

uint32_t pick_k(uint64_t n, uint64_t V, uint32_t target) {
    if (n == 0) return kMaxLocalBits;
    const double r = (double)target * (double)V / (double)n;
    uint32_t k = 0;
    while (k < kMaxLocalBits && (double)(1ull << (k + 1)) <= r) ++k;
    const uint32_t kv = log2_ceil(V);
    return k > kv ? kv : k;
}

}  // namespace

// ------------------------------------------------------------------- plan ---

struct BatchPlanBase {
    virtual ~BatchPlanBase() {}
};

template <typename Key>
struct BatchPlan : BatchPlanBase {
    uint32_t T = 0;
    uint32_t target = 2048;
    uint32_t tiles = 0, bins = 0, qtiles = 0;
    uint32_t max_b1 = 0, max_k = 0;
    uint64_t mat_entries = 0, ws_keys = 0;
    bool build = true;  // false: probe existing tables only
    bool any_order = false;  // order inside a bucket unspecified
    uint32_t part_items = kPartItemsChoices[0];  // keys per partition thread
    ProbeShape probe = kProbeShapes[0];          // probe workgroup shape
    uint32_t part_tile() const { return kPartThreads * part_items; }
    uint32_t probe_tile() const { return probe.threads * probe.items; }
    std::vector<BTable<Key>> host;
    std::vector<uint32_t> tile_pre, bin_pre, qtile_pre;
    // device memory (one block, owned or lent by the caller)
    void* d_block = nullptr;
    bool owns_block = false;
    BTable<Key>* d_tabs = nullptr;
    uint32_t* d_pre = nullptr;  // tile, bin, qtile prefixes
    uint32_t* d_mat = nullptr;
    Key* d_rkeys = nullptr;
    uint32_t* d_rids = nullptr;
    uint32_t* d_heavy = nullptr;  // [bins] list + [1] count
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~BatchPlan() override { release(); }
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        if (owns_block && d_block) (void)hipFree(d_block);
        d_block = nullptr;
        owns_block = false;
    }

    // device bytes of descriptors, prefixes and workspace; carve when base set
    size_t carve(void* base) {
        Carver c(base);
        d_tabs = c.take<BTable<Key>>(T ? T : 1);
        d_pre = c.take<uint32_t>(3 * ((size_t)T + 1));
        d_mat = c.take<uint32_t>(mat_entries ? mat_entries : 1);
        d_rkeys = c.take<Key>(ws_keys ? ws_keys : 1);
        d_rids = c.take<uint32_t>(ws_keys ? ws_keys : 1);
        d_heavy = c.take<uint32_t>((size_t)bins + 1);
        d_block = base;
        return c.off + 256;
    }
    // host image of the descriptors and prefixes, as copied to the device
    size_t host_image_bytes() const { return sizeof(BTable<Key>) * T + 4 * 3 * ((size_t)T + 1); }
    void host_image(void* dst) const {
        char* p = (char*)dst;
        std::memcpy(p, host.data(), sizeof(BTable<Key>) * T);
        p += sizeof(BTable<Key>) * T;
        std::memcpy(p, tile_pre.data(), 4 * (T + 1));
        std::memcpy(p + 4 * (T + 1), bin_pre.data(), 4 * (T + 1));
        std::memcpy(p + 8 * (T + 1), qtile_pre.data(), 4 * (T + 1));
    }
    hipError_t copy_image_async(const void* pinned, hipStream_t s) {
        HG_TRY(hipMemcpyAsync(d_tabs, pinned, sizeof(BTable<Key>) * T, hipMemcpyHostToDevice, s));
        return hipMemcpyAsync(d_pre, (const char*)pinned + sizeof(BTable<Key>) * T,
                              4 * 3 * ((size_t)T + 1), hipMemcpyHostToDevice, s);
    }

    // probe-only layout over existing tables (used by the server to merge
    // small probes into one launch)
    void layout_probe(const std::vector<BTable<Key>>& tabs) {
        build = false;
        T = (uint32_t)tabs.size();
        host = tabs;
        tile_pre.assign(T + 1, 0);
        bin_pre.assign(T + 1, 0);
        qtile_pre.assign(T + 1, 0);
        uint64_t qt = 0;
        for (uint32_t i = 0; i < T; ++i) {
            qtile_pre[i] = (uint32_t)qt;
            qt += ceil_div(host[i].m, probe_tile());
        }
        qtile_pre[T] = (uint32_t)qt;
        tiles = bins = 0;
        qtiles = (uint32_t)qt;
        mat_entries = ws_keys = 0;
    }

    // lay out every table for bin-size target `tgt` (host only)
    hg_status layout(const hg_batch_item* items, uint32_t count, uint32_t tgt) {
        build = true;
        T = count;
        target = tgt;
        host.assign(count, BTable<Key>{});
        tile_pre.assign(count + 1, 0);
        bin_pre.assign(count + 1, 0);
        qtile_pre.assign(count + 1, 0);
        uint64_t tiles64 = 0, bins64 = 0, qt64 = 0, mat64 = 0, keys64 = 0;
        max_b1 = 0;
        max_k = 0;
        for (uint32_t i = 0; i < count; ++i) {
            const hg_batch_item& it = items[i];
            BTable<Key>& tb = host[i];
            tb.keys = (const Key*)it.d_keys;
            tb.queries = (const Key*)it.d_queries;
            tb.offsets = it.d_offsets;
            tb.ids = it.d_ids;
            tb.ekeys = (Key*)it.d_ekeys;
            tb.counts = it.d_counts;
            tb.hp = KeyTraits<Key>::make(it.hash_range, it.seed);
            tb.n = (uint32_t)it.n;
            tb.m = (uint32_t)it.m;
            tb.V = (uint32_t)it.hash_range;
            uint32_t k = pick_k(it.n, it.hash_range, tgt);
            uint32_t bins = (uint32_t)ceil_div(it.hash_range, 1ull << k);
            uint32_t bits = log2_ceil(bins);
            while (bits > kMaxDigitBits && k < kMaxLocalBits) {
                ++k;
                bins = (uint32_t)ceil_div(it.hash_range, 1ull << k);
                bits = log2_ceil(bins);
            }
            if (bits > kMaxDigitBits) return HG_ERR_INVALID_ARG;
            tb.k = k;
            tb.bins = bins;
            if (it.n == 0) {
                tb.kind = kEmpty;
            } else if (bins == 1 && it.n <= light_cap<Key>()) {
                tb.kind = kDirect;
            } else {
                tb.kind = kPartitioned;
                tb.b1 = bits;
                tb.ntiles = (uint32_t)ceil_div(it.n, part_tile());
                tb.mat_base = (uint32_t)mat64;
                tb.key_base = (uint32_t)keys64;
                mat64 += (uint64_t)tb.ntiles << bits;
                keys64 += it.n;
                if (bits > max_b1) max_b1 = bits;
            }
            if (k > max_k) max_k = k;
            tile_pre[i] = (uint32_t)tiles64;
            bin_pre[i] = (uint32_t)bins64;
            qtile_pre[i] = (uint32_t)qt64;
            tiles64 += tb.ntiles;
            bins64 += bins;
            qt64 += ceil_div(it.m, probe_tile());
        }
        tile_pre[count] = (uint32_t)tiles64;
        bin_pre[count] = (uint32_t)bins64;
        qtile_pre[count] = (uint32_t)qt64;
        if (tiles64 > 0x7fffffffull || bins64 > 0x7fffffffull || qt64 > 0x7fffffffull ||
            mat64 > 0xffffffffull || keys64 > 0xffffffffull)
            return HG_ERR_INVALID_ARG;
        tiles = (uint32_t)tiles64;
        bins = (uint32_t)bins64;
        qtiles = (uint32_t)qt64;
        mat_entries = mat64;
        ws_keys = keys64;
        return HG_OK;
    }

    // owned device memory, synchronous upload (graph plans)
    hipError_t upload() {
        void* base = nullptr;
        HG_TRY(hipMalloc(&base, carve(nullptr)));
        carve(base);
        owns_block = true;
        std::vector<char> img(host_image_bytes());
        host_image(img.data());
        HG_TRY(hipMemcpy(d_tabs, img.data(), sizeof(BTable<Key>) * T, hipMemcpyHostToDevice));
        return hipMemcpy(d_pre, img.data() + sizeof(BTable<Key>) * T, 4 * 3 * ((size_t)T + 1),
                         hipMemcpyHostToDevice);
    }

    // the whole run, enqueued on s (also used inside stream capture)
    hipError_t enqueue(hipStream_t s) {
        BPrefix pre{d_pre, d_pre + (T + 1), d_pre + 2 * (T + 1), T};
        uint32_t* heavy_count = d_heavy + bins;
        if (build) {
            hipLaunchKernelGGL(k_bclear, dim3(1), dim3(64), 0, s, heavy_count);
            HG_TRY(hipGetLastError());
        }
        if (tiles) {
            HG_TRY(part_items == 8 ? enqueue_partition<8>(pre, s) : enqueue_partition<16>(pre, s));
        }
        if (bins) {
            hipLaunchKernelGGL(k_blocal<Key>, dim3(bins), dim3(kLocalThreads),
                               light_smem<Key>(max_k), s, (const BTable<Key>*)d_tabs, pre, bins,
                               (const uint32_t*)d_mat, (const Key*)d_rkeys,
                               (const uint32_t*)d_rids, d_heavy, heavy_count, any_order);
            HG_TRY(hipGetLastError());
            const uint32_t hgrid = bins < 256 ? bins : 256;
            hipLaunchKernelGGL(k_bheavy<Key>, dim3(hgrid), dim3(kLocalThreads),
                               heavy_smem<Key>(max_k), s, (const BTable<Key>*)d_tabs, pre,
                               (const uint32_t*)d_mat, (const Key*)d_rkeys,
                               (const uint32_t*)d_rids, (const uint32_t*)d_heavy,
                               (const uint32_t*)heavy_count);
            HG_TRY(hipGetLastError());
        }
        if (qtiles) HG_TRY(enqueue_probe(pre, s));
        return hipSuccess;
    }

    template <int IT>
    hipError_t enqueue_partition(const BPrefix& pre, hipStream_t s) {
        const uint32_t grid = (uint32_t)(8 * ceil_div(tiles, 8));
        hipLaunchKernelGGL((k_bhist<Key, IT>), dim3(grid), dim3(kPartThreads), (4u << max_b1), s,
                           (const BTable<Key>*)d_tabs, pre, tiles, d_mat);
        HG_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_bcolscan<Key>, dim3(T), dim3(256), 0, s, (const BTable<Key>*)d_tabs,
                           d_mat);
        HG_TRY(hipGetLastError());
        const size_t smem = part_smem_bytes(sizeof(Key), max_b1, kPartThreads * IT);
        if (any_order)
            hipLaunchKernelGGL((k_bpart<Key, false, IT>), dim3(grid), dim3(kPartThreads), smem, s,
                               (const BTable<Key>*)d_tabs, pre, tiles, (const uint32_t*)d_mat,
                               d_rkeys, d_rids);
        else
            hipLaunchKernelGGL((k_bpart<Key, true, IT>), dim3(grid), dim3(kPartThreads), smem, s,
                               (const BTable<Key>*)d_tabs, pre, tiles, (const uint32_t*)d_mat,
                               d_rkeys, d_rids);
        return hipGetLastError();
    }

    hipError_t enqueue_probe(const BPrefix& pre, hipStream_t s) {
        const BTable<Key>* tabs = d_tabs;
        const uint32_t qgrid = (uint32_t)(8 * ceil_div(qtiles, 8));
#define HG_BPROBE(TH, IT)                                                                  \
    if (probe.threads == TH && probe.items == IT) {                                        \
        hipLaunchKernelGGL((k_bprobe<Key, TH, IT>), dim3(qgrid), dim3(TH), 0, s, tabs, pre, \
                           qtiles);                                                        \
        return hipGetLastError();                                                          \
    }
        HG_BPROBE(256, 4)
        HG_BPROBE(256, 8)
        HG_BPROBE(512, 2)
        HG_BPROBE(128, 8)
#undef HG_BPROBE
        return hipErrorInvalidValue;
    }

    hipError_t capture() {
        hipStream_t cs;
        HG_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e1 = enqueue(cs);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(cs, &g);
            e = e1 != hipSuccess ? e1 : e2;
            if (e == hipSuccess) {
                graph = g;
                e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
        (void)hipStreamDestroy(cs);
        return e;
    }
};

template <typename Key>
static hipError_t set_batch_smem() {
    static std::atomic<uint64_t> done{0};
    return once_per_device(done, [] {
        const int lim = 160 * 1024;
        HG_TRY(hipFuncSetAttribute((const void*)k_bpart<Key, true, 16>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_bpart<Key, false, 16>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_bpart<Key, true, 8>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_bpart<Key, false, 8>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_bhist<Key, 16>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_bhist<Key, 8>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_blocal<Key>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_bheavy<Key>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        return hipSuccess;
    });
}

// A batch plan's tunable launch configuration.
struct BConfig {
    uint32_t target;      // keys per final bin (sets the partition width)
    uint32_t part_items;  // keys per thread of a partition tile
    ProbeShape probe;     // probe workgroup: threads x queries per thread
};

// Autotuning cache: (tables, total keys, total queries, key bits, any order)
// -> the configuration the tuner chose.
static std::mutex g_tune_mu;
static std::map<std::tuple<uint32_t, uint64_t, uint64_t, int, bool>, BConfig> g_tune;

}  // namespace hg

using namespace hg;

struct hg_batch {
    int key_bits = 32;
    BatchPlanBase* plan = nullptr;
    uint32_t target = 0;
    uint32_t part_items = 0;
    uint32_t probe_threads = 0, probe_items = 0;
};

namespace {

hg_status hstat(hipError_t e) {
    if (e == hipSuccess) return HG_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return HG_ERR_OOM;
    return HG_ERR_DEVICE;
}

// Lay out, upload and capture one candidate plan.
template <typename Key>
hg_status make_plan(const hg_batch_item* items, uint32_t count, bool any_order, const BConfig& c,
                    BatchPlan<Key>** out) {
    BatchPlan<Key>* p = new (std::nothrow) BatchPlan<Key>();
    if (!p) return HG_ERR_OOM;
    p->any_order = any_order;
    p->part_items = c.part_items;
    p->probe = c.probe;
    hg_status st = p->layout(items, count, c.target);
    if (st == HG_OK) st = hstat(p->upload());
    if (st == HG_OK) st = hstat(p->capture());
    if (st != HG_OK) {
        delete p;
        return st;
    }
    *out = p;
    return HG_OK;
}

// Time two replays of a captured plan (after one warm-up replay).
template <typename Key>
hg_status time_plan(BatchPlan<Key>* p, float* ms) {
    hipStream_t ts = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t te = hipStreamCreateWithFlags(&ts, hipStreamNonBlocking);
    if (te == hipSuccess) te = hipEventCreate(&e0);
    if (te == hipSuccess) te = hipEventCreate(&e1);
    if (te == hipSuccess) te = hipGraphLaunch(p->exec, ts);
    if (te == hipSuccess) te = hipEventRecord(e0, ts);
    for (int r = 0; r < 2 && te == hipSuccess; ++r) te = hipGraphLaunch(p->exec, ts);
    if (te == hipSuccess) te = hipEventRecord(e1, ts);
    if (te == hipSuccess) te = hipEventSynchronize(e1);
    if (te == hipSuccess) te = hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ts) (void)hipStreamDestroy(ts);
    return hstat(te);
}

bool probe_shape_ok(uint32_t threads, uint32_t items) {
    for (const ProbeShape& ps : kProbeShapes)
        if (ps.threads == threads && ps.items == items) return true;
    return false;
}

// The tuner searches one dimension at a time over the batch itself: the bin
// target (partition width) with the default tile shapes, then the partition
// tile's keys per thread at the best target, then the probe workgroup shape.
// Each step keeps the fastest graph; a dimension fixed in opts is not
// searched.  The result is cached per batch shape.
template <typename Key>
hg_status create_plan(const hg_batch_item* items, uint32_t count, const hg_batch_opts* opts,
                      hg_batch* b) {
    hipError_t e = set_batch_smem<Key>();
    if (e != hipSuccess) return hstat(e);
    uint64_t tn = 0, tm = 0;
    for (uint32_t i = 0; i < count; ++i) {
        tn += items[i].n;
        tm += items[i].m;
    }
    const int kb = (int)sizeof(Key) * 8;
    const bool any_order = opts && opts->any_order;
    const bool autotune = !opts || opts->autotune != 0;
    const bool fix_target = opts && opts->bin_target;
    const bool fix_part = opts && opts->part_items;
    const bool fix_probe = opts && opts->probe_threads;
    BConfig cfg{fix_target ? opts->bin_target : 2048u,
                fix_part ? opts->part_items : kPartItemsChoices[0],
                fix_probe ? ProbeShape{opts->probe_threads, opts->probe_items} : kProbeShapes[0]};
    const auto key = std::make_tuple(count, tn, tm, kb, any_order);
    bool tune = autotune && !(fix_target && fix_part && fix_probe);
    if (tune) {
        // a batch of the same shape tuned before keeps its choice
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            if (!fix_target) cfg.target = it->second.target;
            if (!fix_part) cfg.part_items = it->second.part_items;
            if (!fix_probe) cfg.probe = it->second.probe;
            tune = false;
        }
    }
    BatchPlan<Key>* best = nullptr;
    if (!tune) {
        hg_status st = make_plan<Key>(items, count, any_order, cfg, &best);
        if (st != HG_OK) return st;
    } else {
        float best_ms = 0.f;
        // candidate configurations of one dimension, timed against the best
        auto search = [&](const std::vector<BConfig>& cands) -> hg_status {
            for (const BConfig& c : cands) {
                BatchPlan<Key>* p = nullptr;
                hg_status st = make_plan<Key>(items, count, any_order, c, &p);
                float ms = 0.f;
                if (st == HG_OK) st = time_plan<Key>(p, &ms);
                if (st != HG_OK) {
                    delete p;
                    return st;
                }
                if (!best || ms < best_ms) {
                    delete best;
                    best = p;
                    best_ms = ms;
                    cfg = c;
                } else {
                    delete p;
                }
            }
            return HG_OK;
        };
        std::vector<BConfig> cands;
        if (fix_target) {
            cands.push_back(cfg);
        } else {
            // a light bin holds up to light_cap<Key>() keys (4608 / 3072)
            for (uint32_t t : {1024u, 2048u, 4096u})
                if (t < light_cap<Key>()) cands.push_back(BConfig{t, cfg.part_items, cfg.probe});
        }
        hg_status st = search(cands);
        if (st == HG_OK && !fix_part) {
            cands.clear();
            for (uint32_t it : kPartItemsChoices)
                if (it != cfg.part_items) cands.push_back(BConfig{cfg.target, it, cfg.probe});
            st = search(cands);
        }
        if (st == HG_OK && !fix_probe) {
            cands.clear();
            for (const ProbeShape& ps : kProbeShapes)
                if (ps.threads != cfg.probe.threads || ps.items != cfg.probe.items)
                    cands.push_back(BConfig{cfg.target, cfg.part_items, ps});
            st = search(cands);
        }
        if (st != HG_OK) {
            delete best;
            return st;
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = cfg;
    }
    b->plan = best;
    b->target = best->target;
    b->part_items = best->part_items;
    b->probe_threads = best->probe.threads;
    b->probe_items = best->probe.items;
    return HG_OK;
}

}  // namespace

extern "C" {

hg_status hg_batch_create(const hg_batch_item* items, uint32_t count, int key_bits,
                          const hg_batch_opts* opts, hg_batch** out) {
    if (!out || (count && !items) || (key_bits != 32 && key_bits != 64)) return HG_ERR_INVALID_ARG;
    if (opts && ((opts->part_items && opts->part_items != 8 && opts->part_items != 16) ||
                 (!opts->probe_threads != !opts->probe_items) ||
                 (opts->probe_threads && !probe_shape_ok(opts->probe_threads, opts->probe_items))))
        return HG_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < count; ++i) {
        const hg_batch_item& it = items[i];
        if (it.hash_range < 1 || it.hash_range > 0xffffffffull || it.n > 0xffffffffull ||
            it.m > 0xffffffffull)
            return HG_ERR_INVALID_ARG;
        if ((it.n && (!it.d_keys || !it.d_ids || !it.d_ekeys)) || !it.d_offsets ||
            (it.m && (!it.d_queries || !it.d_counts)))
            return HG_ERR_INVALID_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return HG_ERR_DEVICE;
    hg_batch* b = new (std::nothrow) hg_batch();
    if (!b) return HG_ERR_OOM;
    b->key_bits = key_bits;
    hg_status st = key_bits == 32 ? create_plan<uint32_t>(items, count, opts, b)
                                  : create_plan<uint64_t>(items, count, opts, b);
    if (st != HG_OK) {
        delete b;
        return st;
    }
    *out = b;
    return HG_OK;
}

hg_status hg_batch_run(hg_batch* b, hipStream_t stream) {
    if (!b || !b->plan) return HG_ERR_INVALID_ARG;
    hipGraphExec_t exec = b->key_bits == 32 ? ((BatchPlan<uint32_t>*)b->plan)->exec
                                            : ((BatchPlan<uint64_t>*)b->plan)->exec;
    return hstat(hipGraphLaunch(exec, stream));
}

hg_status hg_batch_config(const hg_batch* b, hg_batch_opts* out) {
    if (!b || !b->plan || !out) return HG_ERR_INVALID_ARG;
    const bool any_order = b->key_bits == 32 ? ((BatchPlan<uint32_t>*)b->plan)->any_order
                                             : ((BatchPlan<uint64_t>*)b->plan)->any_order;
    *out = hg_batch_opts{};
    out->autotune = 0;
    out->bin_target = b->target;
    out->any_order = any_order ? 1u : 0u;
    out->part_items = b->part_items;
    out->probe_threads = b->probe_threads;
    out->probe_items = b->probe_items;
    return HG_OK;
}

hg_status hg_batch_info(const hg_batch* b, uint32_t* bin_target, uint64_t* workspace_bytes) {
    if (!b || !b->plan) return HG_ERR_INVALID_ARG;
    if (bin_target) *bin_target = b->target;
    if (workspace_bytes) {
        if (b->key_bits == 32) {
            auto* p = (BatchPlan<uint32_t>*)b->plan;
            *workspace_bytes = p->mat_entries * 4 + p->ws_keys * 8;
        } else {
            auto* p = (BatchPlan<uint64_t>*)b->plan;
            *workspace_bytes = p->mat_entries * 4 + p->ws_keys * 12;
        }
    }
    return HG_OK;
}

void hg_batch_free(hg_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    delete b->plan;
    delete b;
}

}  // extern "C"

// ===================================================================== serving
//
// A request loop on a host thread.  Build and probe requests are queued by
// hg_server_submit_*; the loop admits them onto a few HIP streams (default
// priority) as launch slots and memory allow, so work of different requests
// overlaps on the device.  Small requests that are pending together are
// merged into one launch of the batched kernels (continuous batching):
// several small builds become one batched build, several small probes one
// batched probe.  Tables stay resident in HBM until evicted; admission keeps
// resident tables plus in-flight workspace under a byte budget, evicting the
// least recently used tables that no pending or running request uses.
// Latency is measured from submission to the moment a worker sees the
// request's completion event.  Several worker threads (two by default) run
// the loop, each launching on its own share of the streams; they hold the
// server's lock only for bookkeeping (choosing and accounting a launch,
// taking pooled events and pinned buffers, finishing requests): device
// allocations, kernel launches and event polls run with it released, so
// neither submissions nor the other workers wait for the device API.  Each
// table is one device allocation carved into its arrays.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

namespace hg {
namespace srv {

using Clock = std::chrono::steady_clock;

struct STable {
    int key_bits = 32;
    uint64_t n = 0, V = 0, seed = 0;
    void* block = nullptr;  // one device allocation holding every array below
    uint32_t* offsets = nullptr;
    uint32_t* ids = nullptr;
    void* keys = nullptr;
    uint4* head = nullptr;   // probe index (tables built by a launch of their own)
    RunsDev runs{};          // key runs of long buckets (with head)
    bool has_index = false;
    uint64_t bytes = 0;
    uint64_t last_use = 0;
    int pins = 0;            // requests (its build, pending probes) that need it
    hipEvent_t ready = nullptr;
    bool enqueued = false;   // build launched
    bool built = false;      // build completed
    bool failed = false;
    bool accounted = false;  // bytes counted in the server's resident total
    int stream = -1;         // stream of the build
};

struct SReq {
    int kind = 0;  // 0 build, 1 probe
    uint64_t table = 0;
    const void* data = nullptr;
    uint64_t count = 0;
    int key_bits = 32;
    uint32_t* counts = nullptr;
    double t_arrive = 0, t_done = 0;
    hg_status status = HG_OK;
    bool done = false;
    bool keep = true;  // record kept after completion until waited on or drained
};

struct Launch {
    std::vector<uint64_t> reqs;
    uint64_t seq = 0;  // unique per launch (events are pooled and reused)
    hipEvent_t ev = nullptr;
    int stream = 0;
    void* transient = nullptr;
    uint64_t transient_bytes = 0;
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
};

struct Server {
    hg_server_opts o{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, SReq> reqs;
    std::unordered_map<uint64_t, STable> tables;
    std::vector<Launch> inflight;
    uint32_t admitting = 0;  // groups taken off `pending` whose launch is not yet in `inflight`
    std::vector<hipStream_t> streams;
    std::vector<std::pair<void*, size_t>> pinned_free;
    std::vector<hipEvent_t> event_pool;
    uint64_t resident = 0, transient = 0, peak = 0, clock = 0;
    uint64_t next_id = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<uint32_t> worker_next;  // per worker: its next stream
    uint64_t next_seq = 1;
    // statistics
    // latencies of the last kLatKeep completed requests (a ring once full)
    static constexpr size_t kLatKeep = size_t(1) << 20;
    std::vector<double> lat_ms;
    size_t lat_next = 0;
    uint64_t completed = 0, failed = 0, rejected = 0, evictions = 0, launches = 0, merged = 0,
             keys = 0;
    double first_arrive = -1, last_done = 0;
    Clock::time_point t0 = Clock::now();

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    hipEvent_t take_event() {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
        return e;
    }

    void* take_pinned(size_t bytes) {
        for (size_t i = 0; i < pinned_free.size(); ++i)
            if (pinned_free[i].second >= bytes) {
                void* p = pinned_free[i].first;
                pinned_free.erase(pinned_free.begin() + i);
                return p;
            }
        void* p = nullptr;
        size_t sz = bytes < 65536 ? 65536 : bytes;
        if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) return nullptr;
        pinned_sizes[p] = sz;
        return p;
    }
    std::unordered_map<void*, size_t> pinned_sizes;

    // device bytes of a table; with the probe index also 16 per bucket and the
    // key-run arrays (key, end, kperm) per entry
    static uint64_t table_bytes(uint64_t n, uint64_t V, int kb, bool index) {
        const uint64_t nn = n ? n : 1;
        return (V + 1) * 4 + nn * (4 + (uint64_t)kb / 8) +
               (index ? V * 16 + nn * ((uint64_t)kb / 8 + 8) : 0);
    }

    void free_table(STable& t, hipStream_t s) {
        if (t.block) (void)hipFreeAsync(t.block, s);
        t.block = nullptr;
    }

    // Carve a table's arrays out of one block (sizes first when base is null).
    static size_t carve_table(STable& t, void* base) {
        Carver c(base);
        const uint64_t nn = t.n ? t.n : 1, ks = (uint64_t)(t.key_bits / 8);
        t.offsets = c.take<uint32_t>(t.V + 1);
        t.ids = c.take<uint32_t>(nn);
        t.keys = c.take<char>(nn * ks);
        if (t.has_index) {
            t.head = c.take<uint4>(t.V);
            t.runs.run_key = c.take<char>(nn * ks);
            t.runs.run_end = c.take<uint32_t>(nn);
            t.runs.kperm = c.take<uint32_t>(nn);
        }
        return c.off + 256;
    }

    bool evict_for(uint64_t need) {
        while (resident + transient + need > o.budget_bytes) {
            uint64_t victim = 0, best = ~0ull;
            for (auto& kv : tables) {
                const STable& t = kv.second;
                if (t.pins == 0 && t.built && t.last_use < best) {
                    best = t.last_use;
                    victim = kv.first;
                }
            }
            if (!victim) return false;
            drop_table(tables.find(victim));
            ++evictions;
        }
        return true;
    }

    // Complete a request (under the lock).  A record that no caller can
    // wait on is released here; a table whose build failed is released once
    // no pending request names it.
    void finish_req(uint64_t rid, hg_status st, double t) {
        SReq& r = reqs[rid];
        r.status = st;
        r.done = true;
        r.t_done = t;
        auto it = tables.find(r.table);
        if (it != tables.end()) {
            STable& tb = it->second;
            tb.pins -= 1;
            if (r.kind == 0) {
                tb.built = st == HG_OK;
                tb.failed = st != HG_OK;
            }
            tb.last_use = ++clock;
            if (tb.failed && tb.pins == 0) drop_table(it);
        }
        if (st == HG_OK) {
            ++completed;
            keys += r.count;
            const double ms = (t - r.t_arrive) * 1e3;
            if (lat_ms.size() < kLatKeep) lat_ms.push_back(ms);
            else lat_ms[lat_next++ % kLatKeep] = ms;
            if (t > last_done) last_done = t;
        } else {
            ++failed;
        }
        if (!r.keep) reqs.erase(rid);
    }

    // Free a table's memory and forget it (under the lock; no request may
    // still need it).
    void drop_table(std::unordered_map<uint64_t, STable>::iterator it) {
        STable& t = it->second;
        free_table(t, streams[t.stream >= 0 ? t.stream : 0]);
        if (t.ready) event_pool.push_back(t.ready);
        if (t.accounted) resident -= t.bytes;
        tables.erase(it);
    }

    // Finish the launches whose events have completed.  The events are
    // polled with the lock released, from a snapshot taken under it; a
    // launch is finished (under the lock) only if it is still in flight, so
    // several workers may retire at once.  The launches' workspace is
    // released after the lock is dropped again.
    void retire(std::unique_lock<std::mutex>& lk) {
        if (inflight.empty()) return;
        std::vector<std::pair<uint64_t, hipEvent_t>> snap;
        snap.reserve(inflight.size());
        for (const Launch& L : inflight) snap.push_back({L.seq, L.ev});
        std::vector<std::pair<uint64_t, hipError_t>> done;
        lk.unlock();
        for (auto& x : snap) {
            const hipError_t q = hipEventQuery(x.second);
            if (q != hipErrorNotReady) done.push_back({x.first, q});
        }
        lk.lock();
        if (done.empty()) return;
        const double t = now();
        std::vector<std::pair<void*, int>> frees;
        std::vector<Launch> keep;
        keep.reserve(inflight.size());
        for (Launch& L : inflight) {
            const hipError_t* q = nullptr;
            for (auto& d : done)
                if (d.first == L.seq) q = &d.second;
            if (!q) {
                keep.push_back(L);
                continue;
            }
            const hg_status st = *q == hipSuccess ? HG_OK : HG_ERR_DEVICE;
            for (uint64_t rid : L.reqs) finish_req(rid, st, t);
            if (L.transient) {
                frees.push_back({L.transient, L.stream});
                transient -= L.transient_bytes;
            }
            if (L.pinned) pinned_free.push_back({L.pinned, pinned_sizes[L.pinned]});
            event_pool.push_back(L.ev);
        }
        inflight.swap(keep);
        cv_done.notify_all();
        if (frees.empty()) return;
        lk.unlock();
        for (auto& f : frees) (void)hipFreeAsync(f.first, streams[f.second]);
        lk.lock();
    }

    bool small(const SReq& r) const { return r.count <= o.merge_keys; }

    // Start the oldest pending request, merged with other pending requests
    // of the same kind and key width when they are small.  Returns false if
    // it has to wait for memory.
    bool admit_one(std::unique_lock<std::mutex>& lk, uint32_t wk) {
        const uint64_t rid0 = pending.front();
        SReq& r0 = reqs[rid0];
        std::vector<uint64_t> group{rid0};
        if (small(r0) && o.merge_max > 1) {
            for (size_t j = 1; j < pending.size() && group.size() < o.merge_max; ++j) {
                SReq& r = reqs[pending[j]];
                if (r.kind == r0.kind && r.key_bits == r0.key_bits && small(r)) {
                    if (r.kind == 1) {
                        auto it = tables.find(r.table);
                        if (it == tables.end() || !it->second.enqueued || it->second.failed)
                            continue;
                    }
                    group.push_back(pending[j]);
                }
            }
        }
        // probes: their table must exist and have its build launched
        if (r0.kind == 1) {
            auto it = tables.find(r0.table);
            if (it == tables.end() || it->second.failed) {
                pending.pop_front();
                finish_req(rid0, HG_ERR_NOT_FOUND, now());
                cv_done.notify_all();
                return true;
            }
            if (!it->second.enqueued) return false;  // its build waits for memory
        }
        // memory: new tables (builds) plus workspace
        uint64_t need_tables = 0, ws = 0;
        const int kb = r0.key_bits;
        // merged launches carry descriptors + workspace in one block
        BatchPlan<uint32_t> p32;
        BatchPlan<uint64_t> p64;
        for (;;) {
            need_tables = ws = 0;
            uint64_t merged_ws = 0;
            if (group.size() > 1) {
                if (r0.kind == 0) {
                    std::vector<hg_batch_item> items;
                    for (uint64_t rid : group) {
                        const SReq& r = reqs[rid];
                        const STable& t = tables[r.table];
                        hg_batch_item it{};
                        it.d_keys = r.data;
                        it.n = r.count;
                        it.hash_range = t.V;
                        it.seed = t.seed;
                        items.push_back(it);
                    }
                    // output pointers are filled after allocation
                    const hg_status ls = kb == 32
                        ? p32.layout(items.data(), (uint32_t)items.size(), 2048)
                        : p64.layout(items.data(), (uint32_t)items.size(), 2048);
                    if (ls != HG_OK) group.resize(1);
                    else merged_ws = kb == 32 ? p32.carve(nullptr) : p64.carve(nullptr);
                } else {
                    // probes of built (or launched) tables: descriptors and
                    // prefixes in one workspace block
                    merged_ws = kb == 32 ? layout_merged_probe<uint32_t>(p32, group)
                                         : layout_merged_probe<uint64_t>(p64, group);
                    ws = merged_ws;
                }
            }
            if (r0.kind == 0) {
                // a build of its own writes the probe index and key runs;
                // merged small builds (the batched kernels) do not
                const bool idx = group.size() == 1;
                for (uint64_t rid : group) {
                    STable& t = tables[reqs[rid].table];
                    t.has_index = idx;
                    t.bytes = table_bytes(t.n, t.V, t.key_bits, idx);
                    need_tables += t.bytes;
                }
                ws = idx ? build_ws_bytes(2, r0.count, tables[r0.table].V, kb, 0) : merged_ws;
            }
            const uint64_t need = need_tables + ws;
            if (resident + transient + need <= o.budget_bytes) break;
            // evict least recently used tables only if that makes room
            uint64_t evictable = 0;
            for (auto& kv : tables)
                if (kv.second.pins == 0 && kv.second.built) evictable += kv.second.bytes;
            if (need <= o.budget_bytes && resident + transient - evictable + need <= o.budget_bytes) {
                if (!evict_for(need)) return false;
                break;
            }
            // a merged group that does not fit falls back to its oldest request
            if (group.size() > 1) {
                group.resize(1);
                continue;
            }
            // larger than the whole budget, or nothing running will free
            // memory: reject; otherwise wait for running launches
            if (need > o.budget_bytes || (inflight.empty() && !admitting)) {
                pending.pop_front();
                if (r0.kind == 0) {
                    tables[r0.table].failed = true;
                    ++rejected;
                }
                finish_req(rid0, HG_ERR_BUDGET, now());
                cv_done.notify_all();
                return true;
            }
            return false;
        }
        // remove the group from pending; until its launch is published (or
        // has failed) `admitting` keeps hg_server_drain waiting for it
        for (uint64_t rid : group)
            for (size_t j = 0; j < pending.size(); ++j)
                if (pending[j] == rid) {
                    pending.erase(pending.begin() + j);
                    break;
                }
        ++admitting;
        Launch L;
        L.reqs = group;
        L.seq = next_seq++;
        // worker wk launches on streams wk, wk + workers, ... in turn
        {
            const uint32_t W = (uint32_t)workers.size() ? (uint32_t)workers.size() : 1u;
            const uint32_t per = ((uint32_t)streams.size() + W - 1 - wk) / W;  // >= 1
            L.stream = (int)(wk + W * (worker_next[wk] % per));
            worker_next[wk] += 1;
        }
        hipStream_t s = streams[L.stream];
        // The group's requests and tables are reached through pointers from
        // here on: map nodes do not move when other threads insert, and only
        // this thread erases them.  Memory is accounted before the lock is
        // released, so that statistics and admission see it at once.
        std::vector<SReq*> greq;
        std::vector<STable*> gtab;
        for (uint64_t rid : group) {
            SReq* r = &reqs[rid];
            greq.push_back(r);
            gtab.push_back(&tables[r->table]);
        }
        std::vector<size_t> tbytes;
        if (r0.kind == 0)
            for (STable* t : gtab) {
                tbytes.push_back(carve_table(*t, nullptr));
                resident += t->bytes;
                t->accounted = true;
                t->stream = L.stream;
            }
        if (ws) {
            L.transient_bytes = ws;
            transient += ws;
        }
        if (resident + transient > peak) peak = resident + transient;
        // pooled events and the merged launch's pinned descriptor image are
        // taken here, under the lock
        L.ev = take_event();
        if (r0.kind == 0)
            for (STable* t : gtab)
                if (!t->ready) t->ready = take_event();
        if (group.size() > 1)
            L.pinned = take_pinned(kb == 32 ? p32.host_image_bytes() : p64.host_image_bytes());
        // probes wait for their tables' builds launched on other streams
        std::vector<hipEvent_t> waits;
        if (r0.kind == 1)
            for (STable* t : gtab)
                if (!t->built && t->ready && t->stream != L.stream) waits.push_back(t->ready);
        const SReq rq0 = r0;
        // device work: allocations, launches and events, without the lock
        // (submissions go on meanwhile)
        lk.unlock();
        hipError_t e = hipSuccess;
        if (r0.kind == 0)
            for (size_t i = 0; i < gtab.size() && e == hipSuccess; ++i) {
                STable& t = *gtab[i];
                e = hipMallocAsync(&t.block, tbytes[i], s);
                if (e == hipSuccess) carve_table(t, t.block);
            }
        if (e == hipSuccess && ws) e = hipMallocAsync(&L.transient, ws, s);
        for (size_t i = 0; i < waits.size() && e == hipSuccess; ++i)
            e = hipStreamWaitEvent(s, waits[i], 0);
        if (e == hipSuccess) {
            if (rq0.kind == 0 && group.size() == 1) {
                STable& t = *gtab[0];
                IndexOut ix{};
                ix.head = t.head;
                ix.runs = t.runs;
                e = kb == 32 ? run_build_v2<uint32_t>((const uint32_t*)rq0.data, t.n, t.V, t.seed,
                                                      t.offsets, t.ids, (uint32_t*)t.keys,
                                                      ix, L.transient, 0, true, s)
                             : run_build_v2<uint64_t>((const uint64_t*)rq0.data, t.n, t.V, t.seed,
                                                      t.offsets, t.ids, (uint64_t*)t.keys,
                                                      ix, L.transient, 0, true, s);
            } else if (rq0.kind == 1 && group.size() == 1) {
                const STable& t = *gtab[0];
                TableDev d{t.offsets, t.ids, t.keys, t.n, t.V, t.seed};
                if (t.has_index) {
                    d.head = t.head;
                    d.runs = t.runs;
                }
                e = kb == 32 ? run_probe_counts<uint32_t>(d, (const uint32_t*)rq0.data, rq0.count,
                                                          rq0.counts, nullptr, s)
                             : run_probe_counts<uint64_t>(d, (const uint64_t*)rq0.data, rq0.count,
                                                          rq0.counts, nullptr, s);
            } else {
                e = kb == 32 ? enqueue_merged<uint32_t>(p32, rq0.kind == 0, gtab, L, s)
                             : enqueue_merged<uint64_t>(p64, rq0.kind == 0, gtab, L, s);
            }
        }
        if (e == hipSuccess && rq0.kind == 0)
            for (STable* t : gtab) {
                e = hipEventRecord(t->ready, s);
                if (e != hipSuccess) break;
            }
        if (e == hipSuccess) e = hipEventRecord(L.ev, s);
        if (e != hipSuccess) (void)hipStreamSynchronize(s);
        lk.lock();
        --admitting;
        // other workers admit probes of these tables from now on (their
        // arrays were written before the lock was taken again)
        if (e == hipSuccess && rq0.kind == 0)
            for (STable* t : gtab) t->enqueued = true;
        ++launches;
        if (group.size() > 1) merged += group.size();
        if (e != hipSuccess) {
            for (uint64_t rid : group) finish_req(rid, HG_ERR_DEVICE, now());
            if (L.transient) {
                (void)hipFreeAsync(L.transient, s);
                L.transient = nullptr;
            }
            transient -= L.transient_bytes;
            event_pool.push_back(L.ev);
            if (L.pinned) pinned_free.push_back({L.pinned, pinned_sizes[L.pinned]});
            cv_done.notify_all();
            return true;
        }
        inflight.push_back(L);
        return true;
    }

    // Probe-only layout of a group of small probes (under the lock); returns
    // the workspace bytes of the merged launch.
    template <typename Key>
    size_t layout_merged_probe(BatchPlan<Key>& p, const std::vector<uint64_t>& group) {
        std::vector<BTable<Key>> tabs;
        for (uint64_t rid : group) {
            const SReq& r = reqs[rid];
            const STable& t = tables[r.table];
            BTable<Key> b{};
            b.queries = (const Key*)r.data;
            b.offsets = t.offsets;
            b.ids = t.ids;
            b.ekeys = (Key*)t.keys;
            b.counts = r.counts;
            b.hp = KeyTraits<Key>::make(t.V, t.seed);
            b.n = (uint32_t)t.n;
            b.m = (uint32_t)r.count;
            b.V = (uint32_t)t.V;
            b.kind = kEmpty;
            tabs.push_back(b);
        }
        p.layout_probe(tabs);
        return p.carve(nullptr);
    }

    // A merged launch of the group's builds or probes into the launch's
    // workspace (called without the lock: it reaches the tables only through
    // the pointers given).
    template <typename Key>
    hipError_t enqueue_merged(BatchPlan<Key>& p, bool builds, const std::vector<STable*>& gtab,
                              Launch& L, hipStream_t s) {
        if (builds)
            for (size_t i = 0; i < gtab.size(); ++i) {
                const STable& t = *gtab[i];
                p.host[i].offsets = t.offsets;
                p.host[i].ids = t.ids;
                p.host[i].ekeys = (Key*)t.keys;
            }
        p.carve(L.transient);
        if (!L.pinned) return hipErrorOutOfMemory;
        p.host_image(L.pinned);
        HG_TRY(p.copy_image_async(L.pinned, s));
        return p.enqueue(s);
    }

    void loop(uint32_t wk) {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            retire(lk);
            while (!pending.empty() && inflight.size() < o.max_inflight)
                if (!admit_one(lk, wk)) break;
            if (stop && pending.empty() && inflight.empty()) break;
            if (inflight.empty() && pending.empty())
                cv_work.wait(lk);
            else
                cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
};

}  // namespace srv
}  // namespace hg

struct hg_server {
    hg::srv::Server s;
};

extern "C" {

hg_status hg_server_create(const hg_server_opts* opts, hg_server** out) {
    if (!out) return HG_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return HG_ERR_DEVICE;
    hg_server* h = new (std::nothrow) hg_server();
    if (!h) return HG_ERR_OOM;
    hg::srv::Server& s = h->s;
    if (opts) s.o = *opts;
    if (!s.o.budget_bytes) s.o.budget_bytes = 64ull << 30;
    if (!s.o.streams) s.o.streams = 4;
    if (!s.o.max_inflight) s.o.max_inflight = 8;
    if (!s.o.merge_max) s.o.merge_max = 64;
    if (!s.o.merge_keys) s.o.merge_keys = 1u << 18;
    if (!s.o.workers) s.o.workers = s.o.streams < 2 ? s.o.streams : 2;
    if (s.o.streams > 16 || s.o.max_inflight > 256 || s.o.workers > 8 ||
        s.o.workers > s.o.streams) {
        delete h;
        return HG_ERR_INVALID_ARG;
    }
    (void)hipGetDevice(&s.device);
    hg_status st = HG_OK;
    if (hg::set_batch_smem<uint32_t>() != hipSuccess || hg::set_batch_smem<uint64_t>() != hipSuccess)
        st = HG_ERR_DEVICE;
    for (uint32_t i = 0; i < s.o.streams && st == HG_OK; ++i) {
        hipStream_t q;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) st = HG_ERR_DEVICE;
        else s.streams.push_back(q);
    }
    if (st != HG_OK) {
        for (auto q : s.streams) (void)hipStreamDestroy(q);
        delete h;
        return st;
    }
    s.worker_next.assign(s.o.workers, 0u);
    {
        // workers start under the lock, so that none runs before all exist
        std::lock_guard<std::mutex> lk(s.mu);
        for (uint32_t w = 0; w < s.o.workers; ++w)
            s.workers.emplace_back([&s, w] { s.loop(w); });
    }
    *out = h;
    return HG_OK;
}

hg_status hg_server_submit_build(hg_server* h, const void* d_keys, uint64_t n, int key_bits,
                                 uint64_t hash_range, uint64_t seed, uint64_t* table_id,
                                 uint64_t* request_id) {
    if (!h || !table_id || (key_bits != 32 && key_bits != 64) || hash_range < 1 ||
        hash_range > 0xffffffffull || n > 0xffffffffull || (n && !d_keys))
        return HG_ERR_INVALID_ARG;
    hg::srv::Server& s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    if (s.stop) return HG_ERR_INVALID_ARG;
    const uint64_t tid = s.next_id++, rid = s.next_id++;
    hg::srv::STable& t = s.tables[tid];
    t.key_bits = key_bits;
    t.n = n;
    t.V = hash_range;
    t.seed = seed;
    t.bytes = hg::srv::Server::table_bytes(n, hash_range, key_bits, true);
    t.pins = 1;
    t.last_use = ++s.clock;
    hg::srv::SReq& r = s.reqs[rid];
    r.kind = 0;
    r.table = tid;
    r.data = d_keys;
    r.count = n;
    r.key_bits = key_bits;
    r.keep = request_id != nullptr;
    r.t_arrive = s.now();
    if (s.first_arrive < 0) s.first_arrive = r.t_arrive;
    s.pending.push_back(rid);
    *table_id = tid;
    if (request_id) *request_id = rid;
    s.cv_work.notify_one();
    return HG_OK;
}

hg_status hg_server_submit_probe(hg_server* h, uint64_t table_id, const void* d_queries,
                                 uint64_t m, uint32_t* d_counts, uint64_t* request_id) {
    if (!h || m > 0xffffffffull || (m && (!d_queries || !d_counts))) return HG_ERR_INVALID_ARG;
    hg::srv::Server& s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    if (s.stop) return HG_ERR_INVALID_ARG;
    auto it = s.tables.find(table_id);
    if (it == s.tables.end() || it->second.failed) return HG_ERR_NOT_FOUND;
    it->second.pins += 1;
    it->second.last_use = ++s.clock;
    const uint64_t rid = s.next_id++;
    hg::srv::SReq& r = s.reqs[rid];
    r.kind = 1;
    r.table = table_id;
    r.data = d_queries;
    r.count = m;
    r.key_bits = it->second.key_bits;
    r.counts = d_counts;
    r.keep = request_id != nullptr;
    r.t_arrive = s.now();
    if (s.first_arrive < 0) s.first_arrive = r.t_arrive;
    s.pending.push_back(rid);
    if (request_id) *request_id = rid;
    s.cv_work.notify_one();
    return HG_OK;
}

hg_status hg_server_wait(hg_server* h, uint64_t request_id, hg_status* result) {
    if (!h) return HG_ERR_INVALID_ARG;
    hg::srv::Server& s = h->s;
    std::unique_lock<std::mutex> lk(s.mu);
    if (s.reqs.find(request_id) == s.reqs.end()) return HG_ERR_NOT_FOUND;
    // another waiter (or a drain) may release the record meanwhile
    s.cv_done.wait(lk, [&] {
        auto f = s.reqs.find(request_id);
        return f == s.reqs.end() || f->second.done;
    });
    auto it = s.reqs.find(request_id);
    if (it == s.reqs.end()) return HG_ERR_NOT_FOUND;
    if (result) *result = it->second.status;
    s.reqs.erase(it);
    return HG_OK;
}

hg_status hg_server_drain(hg_server* h) {
    if (!h) return HG_ERR_INVALID_ARG;
    hg::srv::Server& s = h->s;
    std::unique_lock<std::mutex> lk(s.mu);
    s.cv_done.wait(lk, [&] { return s.pending.empty() && s.inflight.empty() && !s.admitting; });
    // every request has completed: release the records
    for (auto it = s.reqs.begin(); it != s.reqs.end();)
        it = it->second.done ? s.reqs.erase(it) : std::next(it);
    s.cv_done.notify_all();
    return HG_OK;
}

hg_status hg_server_table(hg_server* h, uint64_t table_id, hg_table_info* info) {
    if (!h || !info) return HG_ERR_INVALID_ARG;
    hg::srv::Server& s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.tables.find(table_id);
    if (it == s.tables.end() || !it->second.built) return HG_ERR_NOT_FOUND;
    const hg::srv::STable& t = it->second;
    info->d_offsets = t.offsets;
    info->d_ids = t.ids;
    info->d_keys = t.keys;
    info->n = t.n;
    info->hash_range = t.V;
    info->seed = t.seed;
    info->key_bits = t.key_bits;
    info->variant = HG_VARIANT_V2;
    info->device_bytes = t.bytes;
    return HG_OK;
}

hg_status hg_server_export(hg_server* h, uint64_t table_id, uint32_t* d_offsets, uint32_t* d_ids,
                           void* d_keys, hipStream_t stream) {
    if (!h) return HG_ERR_INVALID_ARG;
    hg::srv::Server& s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.tables.find(table_id);
    if (it == s.tables.end() || !it->second.built) return HG_ERR_NOT_FOUND;
    const hg::srv::STable& t = it->second;
    if (t.ready && hipStreamWaitEvent(stream, t.ready, 0) != hipSuccess) return HG_ERR_DEVICE;
    hipError_t e = hipSuccess;
    if (d_offsets)
        e = hipMemcpyAsync(d_offsets, t.offsets, (t.V + 1) * 4, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && d_ids && t.n)
        e = hipMemcpyAsync(d_ids, t.ids, t.n * 4, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && d_keys && t.n)
        e = hipMemcpyAsync(d_keys, t.keys, t.n * (uint64_t)(t.key_bits / 8),
                           hipMemcpyDeviceToDevice, stream);
    // finish the copy before the table can be evicted
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return e == hipSuccess ? HG_OK : HG_ERR_DEVICE;
}

hg_status hg_server_stats_get(hg_server* h, hg_server_stats* out) {
    if (!h || !out) return HG_ERR_INVALID_ARG;
    hg::srv::Server& s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    hg_server_stats r{};
    r.completed = s.completed;
    r.failed = s.failed;
    r.rejected = s.rejected;
    r.evictions = s.evictions;
    r.launches = s.launches;
    r.merged_requests = s.merged;
    r.keys = s.keys;
    std::vector<double> v = s.lat_ms;
    std::sort(v.begin(), v.end());
    if (!v.empty()) {
        auto q = [&](double f) {
            size_t i = (size_t)(f * (double)(v.size() - 1) + 0.5);
            return v[i < v.size() ? i : v.size() - 1];
        };
        r.p50_ms = q(0.50);
        r.p99_ms = q(0.99);
        r.max_ms = v.back();
        double sum = 0;
        for (double x : v) sum += x;
        r.mean_ms = sum / (double)v.size();
    }
    r.busy_s = s.first_arrive >= 0 ? s.last_done - s.first_arrive : 0.0;
    r.resident_bytes = s.resident;
    r.peak_bytes = s.peak;
    uint32_t nt = 0;
    for (auto& kv : s.tables)
        if (kv.second.built) ++nt;
    r.resident_tables = nt;
    r.held_requests = s.reqs.size() > 0xffffffffull ? 0xffffffffu : (uint32_t)s.reqs.size();
    *out = r;
    return HG_OK;
}

hg_status hg_server_reset_stats(hg_server* h) {
    if (!h) return HG_ERR_INVALID_ARG;
    hg::srv::Server& s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    s.lat_ms.clear();
    s.lat_next = 0;
    s.completed = s.failed = s.rejected = s.evictions = s.launches = s.merged = s.keys = 0;
    s.first_arrive = -1;
    s.last_done = 0;
    s.peak = s.resident + s.transient;
    return HG_OK;
}

void hg_server_destroy(hg_server* h) {
    if (!h) return;
    hg::srv::Server& s = h->s;
    {
        std::lock_guard<std::mutex> lk(s.mu);
        s.stop = true;
        s.cv_work.notify_all();
    }
    for (auto& w : s.workers)
        if (w.joinable()) w.join();
    for (auto q : s.streams) (void)hipStreamSynchronize(q);
    for (auto& kv : s.tables) {
        hg::srv::STable& t = kv.second;
        s.free_table(t, s.streams[0]);
        if (t.ready) (void)hipEventDestroy(t.ready);
    }
    for (auto q : s.streams) (void)hipStreamSynchronize(q);
    for (auto e : s.event_pool) (void)hipEventDestroy(e);
    for (auto& p : s.pinned_free) (void)hipHostFree(p.first);
    for (auto q : s.streams) (void)hipStreamDestroy(q);
    delete h;
}

}  // extern "C"
