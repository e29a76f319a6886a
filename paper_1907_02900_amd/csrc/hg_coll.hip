// Build once, intersect many: a collection of key sets, each stored as its own
// HashGraph, and the match counts of many pairs of sets.  Sec. 3.4 notes that
// Probe-New pays for building the second table, a cost that sparse products
// amortise: the table of every row or column is built once and then takes
// part in many intersections.
//
// Layout.  Set s holds keys[set_off[s] .. set_off[s+1]).  Its table has V_s
// buckets, a power of two: the smallest power of two >= max(n_s, 1), times
// 2^range_shift (clamped to [1, 2^31]).  The tables are concatenated: the
// buckets of set s are [bb[s], bb[s+1]) of one offsets array (bb is the
// exclusive scan of V_s) holding absolute edge positions, and set s's entries
// fill [set_off[s], set_off[s+1]) of the shared ids / keys arrays, sorted by
// bucket with ids ascending inside a bucket; ids are positions in the
// concatenated input.  Set s's table is therefore the stable HashGraph of its
// keys with hash range V_s, shifted by set_off[s].
//
// Build.  Sets are packed into windows by weight w_s = max(ceil(4 n_s / 3),
// V_s): every set starting in a window of weight 2048 that weighs at most
// 2048 itself fits, with the window's other such sets, into one LDS bin of at
// most 3072 keys and 4096 buckets, and one workgroup builds them with the V2
// per-bin body; an entry's set is found by a search over the window's set
// starts held in LDS.  Heavier sets are built together by one stable radix
// sort of (global bucket, input position) pairs, so ids stay ascending inside
// a bucket, and each of their buckets' start is a search in the set's sorted
// segment.
//
// Intersections.  For pair q = (i, j) the smaller set is walked in its table's
// order and each of its keys is looked up in the other set's bucket
// (hash & (V - 1)), counting equal keys: the pair's count is the number of
// entry pairs with equal keys, the size of the join of the two sets (Alg. 3
// over the pair of tables).  Work is balanced over all pairs: an exclusive
// scan of the walked sizes maps work items to pairs, each workgroup takes
// 2048 consecutive items and stages its pairs' metadata (walked keys' start,
// looked-up set's buckets) in LDS, so that an item costs an LDS search, its
// walked key and the looked-up bucket; per-item counts are summed per pair
// inside each wave before one atomic add per (wave, pair).

#include "hg_v2_device.h"

namespace hg {

namespace {

using namespace v2dev;

constexpr int kT = 256;
constexpr uint32_t kGroupW = 2048;                // window weight
constexpr uint32_t kGroupBuckets = 2 * kGroupW;   // buckets a window's sets can span
constexpr uint32_t kPairItems = 8;                // work items per thread
constexpr uint32_t kPairChunk = kT * kPairItems;  // work items per workgroup

static_assert(light_cap<uint32_t>() >= 3 * kGroupW / 2 && light_cap<uint64_t>() >= 3 * kGroupW / 2,
              "a window's keys must fit one LDS bin");

uint32_t grid_of(uint64_t n) {
    const uint64_t g = ceil_div(n, kT);
    return (uint32_t)(g ? g : 1);
}

template <typename Key>
__device__ __forceinline__ uint32_t set_hash(Key k, uint64_t seed);
template <>
__device__ __forceinline__ uint32_t set_hash<uint32_t>(uint32_t k, uint64_t seed) {
    return fmix32(k ^ (uint32_t)seed);
}
template <>
__device__ __forceinline__ uint32_t set_hash<uint64_t>(uint64_t k, uint64_t seed) {
    return (uint32_t)fmix64(k ^ seed);
}

// first index i in [0, n) with a[i] >= x (n if none)
template <typename T, typename U>
__device__ __forceinline__ uint64_t lower_bound_dev(const T* a, uint64_t n, U x) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t m = (lo + hi) >> 1;
        if (a[m] < x)
            lo = m + 1;
        else
            hi = m;
    }
    return lo;
}

// last index i in [0, n) with a[i] <= x, for a[0] <= x
template <typename T, typename U>
__device__ __forceinline__ uint64_t last_le(const T* a, uint64_t n, U x) {
    uint64_t lo = 0, hi = n;  // a[lo] <= x, a[hi] > x (hi = n: past the end)
    while (hi - lo > 1) {
        const uint64_t m = (lo + hi) >> 1;
        if (a[m] <= x)
            lo = m;
        else
            hi = m;
    }
    return lo;
}

__device__ __forceinline__ uint32_t set_range(uint32_t n, int shift) {
    const int lg = n <= 1 ? 0 : 32 - __clz(n - 1);  // ceil(log2 n)
    int e = lg + shift;
    e = e < 0 ? 0 : (e > 31 ? 31 : e);
    return 1u << e;
}

// Per set (and a zero entry at index S for the scans' totals): its hash range,
// weight, and its keys / buckets when it is heavier than a window.
__global__ void k_coll_meta(const uint32_t* __restrict__ set_off, uint32_t S, int shift,
                            uint32_t* __restrict__ range, uint32_t* __restrict__ weight,
                            uint32_t* __restrict__ big_n, uint32_t* __restrict__ big_v,
                            uint32_t* __restrict__ bad) {
    const uint64_t s = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (s > S) return;
    if (s == S) {
        range[s] = weight[s] = big_n[s] = big_v[s] = 0;
        if (set_off[0] != 0) *bad = 1;
        return;
    }
    const uint32_t lo = set_off[s], hi = set_off[s + 1];
    if (hi < lo) *bad = 1;
    const uint32_t n = hi >= lo ? hi - lo : 0u;
    const uint32_t V = set_range(n, shift);
    uint64_t w = ((uint64_t)n * 4 + 2) / 3;
    w = w > V ? w : V;
    w = w < (1ull << 31) ? w : (1ull << 31);
    const bool big = w > kGroupW;
    range[s] = V;
    weight[s] = (uint32_t)w;
    big_n[s] = big ? n : 0u;
    big_v[s] = big ? V : 0u;
}

// One workgroup per window: builds the sets (of at most a window's weight)
// that start in it.
template <typename Key>
__global__ __launch_bounds__(kLocalThreads) void k_coll_groups(
    const Key* __restrict__ keys, const uint32_t* __restrict__ set_off,
    const uint64_t* __restrict__ bb, const uint64_t* __restrict__ cw, uint32_t S, uint64_t seed,
    uint32_t* __restrict__ offsets, uint32_t* __restrict__ ids, Key* __restrict__ ekeys,
    uint32_t* __restrict__ bad) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint64_t w0 = (uint64_t)blockIdx.x * kGroupW;
    const uint32_t s0 = (uint32_t)lower_bound_dev(cw, S, w0);
    uint32_t s1 = (uint32_t)lower_bound_dev(cw, S, w0 + kGroupW);
    // a set heavier than a window can only be the last one to start in it
    if (s1 > s0 && cw[s1] - cw[s1 - 1] > kGroupW) --s1;
    if (s1 <= s0) return;
    const uint32_t ns = s1 - s0, key0 = set_off[s0], L = set_off[s1] - key0;
    const uint64_t B0 = bb[s0];
    const uint32_t NBk = (uint32_t)(bb[s1] - B0);
    if (L > light_cap<Key>() || NBk > kGroupBuckets || ns > kGroupBuckets) {  // excluded by the packing
        if (threadIdx.x == 0) *bad = 1;
        return;
    }
    uint16_t* gstart = (uint16_t*)(smem + light_smem<Key>(12));
    uint16_t* gbkt = gstart + kGroupBuckets + 1;
    for (uint32_t i = threadIdx.x; i <= ns; i += kLocalThreads) {
        gstart[i] = (uint16_t)(set_off[s0 + i] - key0);
        gbkt[i] = (uint16_t)(bb[s0 + i] - B0);
    }
    __syncthreads();
    const uint32_t k = NBk <= 1 ? 0u : 32u - __clz(NBk - 1);
    light_bin_body_by<Key>(
        keys + key0, nullptr, key0, L, key0, 0u, k, NBk,
        [&](Key key, uint32_t e) {
            uint32_t a = 0, b = ns;  // the last set of the window starting at or before e
            while (b - a > 1) {
                const uint32_t m = (a + b) >> 1;
                if (gstart[m] <= e)
                    a = m;
                else
                    b = m;
            }
            const uint32_t V = (uint32_t)gbkt[a + 1] - gbkt[a];
            return (uint32_t)gbkt[a] + (set_hash<Key>(key, seed) & (V - 1u));
        },
        offsets + B0, IndexOut{}, ids, ekeys, smem, false);
}

template <typename Key>
size_t groups_smem() {
    return light_smem<Key>(12) + 2 * (kGroupBuckets + 1) * sizeof(uint16_t);
}

// (global bucket, input position) of every entry of the heavy sets, in set order.
template <typename Key>
__global__ void k_big_keys(const Key* __restrict__ keys, const uint32_t* __restrict__ set_off,
                           const uint64_t* __restrict__ bb, const uint64_t* __restrict__ cb,
                           uint32_t S, uint64_t nbk, uint64_t seed, uint32_t* __restrict__ gb,
                           uint32_t* __restrict__ pos) {
    const uint64_t j = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= nbk) return;
    const uint64_t s = last_le(cb, (uint64_t)S + 1, j);
    const uint32_t p = set_off[s] + (uint32_t)(j - cb[s]);
    const uint32_t V = (uint32_t)(bb[s + 1] - bb[s]);
    gb[j] = (uint32_t)(bb[s] + (set_hash<Key>(keys[p], seed) & (V - 1u)));
    pos[j] = p;
}

template <typename Key>
__global__ void k_big_place(const Key* __restrict__ keys, const uint32_t* __restrict__ set_off,
                            const uint64_t* __restrict__ cb, uint32_t S, uint64_t nbk,
                            const uint32_t* __restrict__ pos_sorted, uint32_t* __restrict__ ids,
                            Key* __restrict__ ekeys) {
    const uint64_t j = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= nbk) return;
    const uint64_t s = last_le(cb, (uint64_t)S + 1, j);
    const uint32_t o = set_off[s] + (uint32_t)(j - cb[s]);
    const uint32_t p = pos_sorted[j];
    ekeys[o] = keys[p];
    ids[o] = p;
}

// offsets of every bucket of the heavy sets
__global__ void k_big_offsets(const uint32_t* __restrict__ set_off, const uint64_t* __restrict__ bb,
                              const uint64_t* __restrict__ cb, const uint64_t* __restrict__ cv,
                              uint32_t S, uint64_t nbv, const uint32_t* __restrict__ gb_sorted,
                              uint32_t* __restrict__ offsets) {
    const uint64_t u = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (u >= nbv) return;
    const uint64_t s = last_le(cv, (uint64_t)S + 1, u);
    const uint64_t g = bb[s] + (u - cv[s]);
    const uint64_t n = cb[s + 1] - cb[s];
    offsets[g] = set_off[s] + (uint32_t)lower_bound_dev(gb_sorted + cb[s], n, (uint32_t)g);
}

// ---- intersections ---------------------------------------------------------

struct SetsView {
    const uint32_t* set_off;
    const uint64_t* bb;
    const uint32_t* offsets;
    const void* keys;
    uint32_t S;
};

__global__ void k_pair_work(const uint32_t* __restrict__ pairs, uint64_t Q, SetsView a, SetsView b,
                            uint32_t* __restrict__ work, uint32_t* __restrict__ bad) {
    const uint64_t q = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (q > Q) return;
    if (q == Q) {
        work[q] = 0;
        return;
    }
    const uint32_t i = pairs[2 * q], j = pairs[2 * q + 1];
    if (i >= a.S || j >= b.S) {
        *bad = 1;
        work[q] = 0;
        return;
    }
    const uint32_t ni = a.set_off[i + 1] - a.set_off[i], nj = b.set_off[j + 1] - b.set_off[j];
    work[q] = ni < nj ? ni : nj;
}

constexpr uint32_t kPairMeta = 1024;  // pairs of a workgroup whose metadata LDS holds

template <typename Key>
__global__ __launch_bounds__(kT) void k_pair_count(const uint32_t* __restrict__ pairs,
                                                   const uint64_t* __restrict__ W, uint64_t Q,
                                                   uint64_t T, SetsView a, SetsView b,
                                                   uint64_t seed,
                                                   unsigned long long* __restrict__ counts,
                                                   unsigned long long* __restrict__ partial) {
    __shared__ uint64_t qrange[2];
    __shared__ unsigned long long red[kT / kWave];
    // per pair of the chunk: its first item relative to the chunk (clamped at
    // 0), the walked key index of the chunk's first item (mod 2^32), the
    // looked-up set's first bucket, and its V - 1 with bit 31 set when a's
    // set is the walked one
    __shared__ uint16_t s_w[kPairMeta];
    __shared__ uint32_t s_kpos[kPairMeta], s_tb[kPairMeta], s_vm[kPairMeta];
    const uint64_t base = (uint64_t)blockIdx.x * kPairChunk;
    if (threadIdx.x == 0) {
        const uint64_t last = (base + kPairChunk < T ? base + kPairChunk : T) - 1;
        qrange[0] = last_le(W, Q + 1, base);
        qrange[1] = last_le(W, Q + 1, last);
    }
    __syncthreads();
    const uint64_t qa = qrange[0], nq = qrange[1] - qa + 1;
    const bool staged = nq <= kPairMeta;  // uniform over the workgroup
    if (staged) {
        for (uint32_t j = threadIdx.x; j < nq; j += kT) {
            const uint64_t q = qa + j;
            const uint32_t i = pairs[2 * q], jj = pairs[2 * q + 1];
            const uint32_t ni = a.set_off[i + 1] - a.set_off[i];
            const uint32_t nj = b.set_off[jj + 1] - b.set_off[jj];
            const bool walk_a = ni < nj;
            const uint32_t wstart = walk_a ? a.set_off[i] : b.set_off[jj];
            const uint64_t* obb = walk_a ? b.bb + jj : a.bb + i;
            const uint64_t wq = W[q];
            s_w[j] = (uint16_t)(wq > base ? wq - base : 0);
            s_kpos[j] = wstart + (uint32_t)base - (uint32_t)wq;
            s_tb[j] = (uint32_t)obb[0];
            s_vm[j] = ((uint32_t)(obb[1] - obb[0]) - 1u) | (walk_a ? 0x80000000u : 0u);
        }
        __syncthreads();
    }
    const uint32_t lane = lane_id();
    unsigned long long mine = 0;
    for (uint32_t r = 0; r < kPairItems; ++r) {
        const uint64_t t = base + (uint64_t)r * kT + threadIdx.x;
        uint64_t q = ~0ull;
        unsigned long long c = 0;
        if (t < T) {
            Key key;
            uint64_t g;
            bool walk_a;
            if (staged) {
                const uint32_t rel = (uint32_t)(t - base);
                uint32_t lo = 0, hi = (uint32_t)nq;  // the last pair starting at or before rel
                while (hi - lo > 1) {
                    const uint32_t m = (lo + hi) >> 1;
                    if (s_w[m] <= rel)
                        lo = m;
                    else
                        hi = m;
                }
                q = qa + lo;
                const uint32_t vm = s_vm[lo];
                walk_a = (vm >> 31) != 0;
                key = ((const Key*)(walk_a ? a.keys : b.keys))[s_kpos[lo] + rel];
                g = (uint64_t)s_tb[lo] + (set_hash<Key>(key, seed) & (vm & 0x7fffffffu));
            } else {
                q = qa + last_le(W + qa, nq, t);
                const uint32_t i = pairs[2 * q], j = pairs[2 * q + 1];
                const uint32_t ni = a.set_off[i + 1] - a.set_off[i];
                const uint32_t nj = b.set_off[j + 1] - b.set_off[j];
                walk_a = ni < nj;
                const SetsView& w = walk_a ? a : b;
                const SetsView& o = walk_a ? b : a;
                const uint32_t sw = walk_a ? i : j, so = walk_a ? j : i;
                key = ((const Key*)w.keys)[w.set_off[sw] + (uint32_t)(t - W[q])];
                const uint64_t ob = o.bb[so];
                const uint32_t V = (uint32_t)(o.bb[so + 1] - ob);
                g = ob + (set_hash<Key>(key, seed) & (V - 1u));
            }
            const SetsView& o = walk_a ? b : a;
            const uint32_t lo = o.offsets[g], hi = o.offsets[g + 1];
            const Key* ok = (const Key*)o.keys;
            for (uint32_t p = lo; p < hi; ++p) c += ok[p] == key;
        }
        mine += c;
        if (counts) {
            // q is non-decreasing over the lanes: sum each run of equal q
            unsigned long long v = c;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const unsigned long long ov = __shfl_up(v, d, kWave);
                const uint64_t oq = __shfl_up(q, d, kWave);
                if (lane >= (uint32_t)d && oq == q) v += ov;
            }
            const uint64_t nq_next = __shfl_down(q, 1, kWave);
            const bool tail = lane == kWave - 1 || nq_next != q;
            if (tail && q != ~0ull && v) atomicAdd(counts + q, v);
        }
    }
    // block total, one plain store per workgroup
    unsigned long long s = mine;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) s += __shfl_xor(s, d, kWave);
    if (lane == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long all = 0;
        for (int i = 0; i < kT / kWave; ++i) all += red[i];
        partial[blockIdx.x] = all;
    }
}

__global__ void k_sum_u64(const unsigned long long* __restrict__ v, uint64_t n,
                          unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[1024 / kWave];
    unsigned long long s = 0;
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) s += v[i];
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) s += __shfl_xor(s, d, kWave);
    if (lane_id() == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long all = 0;
        for (uint32_t i = 0; i < blockDim.x / kWave; ++i) all += red[i];
        *out = all;
    }
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <typename Key>
hipError_t set_group_smem() {
    static std::atomic<uint64_t> done{0};
    return once_per_device(done, [] {
        HG_TRY(hipFuncSetAttribute((const void*)k_coll_groups<Key>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)groups_smem<Key>()));
        return hipSuccess;
    });
}

hipError_t copy_to_host(void* h, const void* d, size_t bytes, hipStream_t s) {
    return hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s);
}

// temporary storage of the (bucket, position) radix sort
size_t pair_sort_bytes(uint64_t n) { return n ? sort_pairs_ws_bytes(n) : 0; }

}  // namespace

// ---- host side ---------------------------------------------------------------

// Workspace layouts: one function carves the buffer and, with a null base,
// measures it, so that sizes and pointers always agree.
struct PlanWs {
    uint32_t *range, *weight, *big_n, *big_v, *bad;
    uint64_t *cw, *cb, *cv;
    void* sws;
};

size_t layout_plan(void* base, uint32_t S, PlanWs* w) {
    const uint64_t n = (uint64_t)S + 1;
    Carver c(base);
    w->range = c.take<uint32_t>(n);
    w->weight = c.take<uint32_t>(n);
    w->big_n = c.take<uint32_t>(n);
    w->big_v = c.take<uint32_t>(n);
    w->cw = c.take<uint64_t>(n + 1);
    w->cb = c.take<uint64_t>(n + 1);
    w->cv = c.take<uint64_t>(n + 1);
    w->bad = c.take<uint32_t>(64);
    w->sws = c.take<unsigned char>(scan_ws_bytes(n));
    return c.off;
}

size_t coll_plan_ws_bytes(uint32_t S) {
    PlanWs w;
    return layout_plan(nullptr, S, &w);
}

hipError_t coll_plan(const uint32_t* set_off, uint32_t S, int shift, void* ws, uint64_t* bb,
                     CollPlan* plan, hipStream_t s) {
    const uint64_t n = (uint64_t)S + 1;
    PlanWs w;
    layout_plan(ws, S, &w);
    uint32_t *range = w.range, *weight = w.weight, *big_n = w.big_n, *big_v = w.big_v;
    uint32_t* bad = w.bad;
    void* sws = w.sws;
    plan->cw = w.cw;
    plan->cb = w.cb;
    plan->cv = w.cv;
    HG_TRY(fill_u32(bad, 1, 0u, s));
    HG_PROF("coll_plan", s);
    hipLaunchKernelGGL(k_coll_meta, dim3(grid_of(n)), dim3(kT), 0, s, set_off, S, shift, range,
                       weight, big_n, big_v, bad);
    HG_TRY(hipGetLastError());
    HG_TRY(scan_excl<uint64_t>(range, n, bb, nullptr, sws, s));
    HG_TRY(scan_excl<uint64_t>(weight, n, plan->cw, nullptr, sws, s));
    HG_TRY(scan_excl<uint64_t>(big_n, n, plan->cb, nullptr, sws, s));
    HG_TRY(scan_excl<uint64_t>(big_v, n, plan->cv, nullptr, sws, s));
    uint32_t h_bad = 0, h_n = 0;
    HG_TRY(copy_to_host(&h_bad, bad, 4, s));
    HG_TRY(copy_to_host(&h_n, set_off + S, 4, s));
    HG_TRY(copy_to_host(&plan->buckets, bb + S, 8, s));
    HG_TRY(copy_to_host(&plan->weight, plan->cw + S, 8, s));
    HG_TRY(copy_to_host(&plan->big_keys, plan->cb + S, 8, s));
    HG_TRY(copy_to_host(&plan->big_buckets, plan->cv + S, 8, s));
    HG_TRY(hipStreamSynchronize(s));
    plan->bad = h_bad != 0;
    plan->n = h_n;
    return hipSuccess;
}

struct BuildWs {
    uint32_t *gb, *gb_s, *pos, *pos_s, *bad;
    void* sort_tmp;
};

size_t layout_build(void* base, uint64_t nbk, BuildWs* w) {
    Carver c(base);
    w->gb = c.take<uint32_t>(nbk + 1);
    w->gb_s = c.take<uint32_t>(nbk + 1);
    w->pos = c.take<uint32_t>(nbk + 1);
    w->pos_s = c.take<uint32_t>(nbk + 1);
    w->bad = c.take<uint32_t>(64);
    w->sort_tmp = c.take<unsigned char>(pair_sort_bytes(nbk));
    return c.off;
}

size_t coll_build_ws_bytes(const CollPlan& p, int key_bits) {
    (void)key_bits;
    BuildWs w;
    return layout_build(nullptr, p.big_keys, &w);
}

template <typename Key>
hipError_t run_coll_build(const Key* keys, const uint32_t* set_off, uint32_t S, uint64_t seed,
                          const uint64_t* bb, const CollPlan& p, void* ws, uint32_t* offsets,
                          uint32_t* ids, Key* ekeys, bool* bad_out, hipStream_t s) {
    HG_TRY(set_group_smem<Key>());
    const uint64_t nbk = p.big_keys;
    BuildWs w;
    layout_build(ws, nbk, &w);
    uint32_t *gb = w.gb, *gb_s = w.gb_s, *pos = w.pos, *pos_s = w.pos_s, *bad = w.bad;
    void* sort_tmp = w.sort_tmp;
    HG_TRY(fill_u32(bad, 1, 0u, s));
    HG_TRY(fill_u32(offsets + p.buckets, 1, (uint32_t)p.n, s));
    const uint64_t windows = ceil_div(p.weight, kGroupW);
    if (windows) {
        HG_PROF("coll_groups", s);
        hipLaunchKernelGGL(k_coll_groups<Key>, dim3((uint32_t)windows), dim3(kLocalThreads),
                           groups_smem<Key>(), s, keys, set_off, bb, (const uint64_t*)p.cw, S, seed,
                           offsets, ids, ekeys, bad);
        HG_TRY(hipGetLastError());
    }
    if (nbk) {
        HG_PROF("coll_big", s);
        hipLaunchKernelGGL(k_big_keys<Key>, dim3(grid_of(nbk)), dim3(kT), 0, s, keys, set_off, bb,
                           (const uint64_t*)p.cb, S, nbk, seed, gb, pos);
        HG_TRY(hipGetLastError());
        const uint32_t bits = p.buckets <= 1 ? 1u : 64u - (uint32_t)__builtin_clzll(p.buckets - 1);
        bool alt = false;
        HG_TRY(sort_pairs_u32(gb, pos, gb_s, pos_s, nbk, bits, sort_tmp, &alt, s));
        if (!alt) {  // the sorted pairs are in the first buffers
            std::swap(gb, gb_s);
            std::swap(pos, pos_s);
        }
        hipLaunchKernelGGL(k_big_place<Key>, dim3(grid_of(nbk)), dim3(kT), 0, s, keys, set_off,
                           (const uint64_t*)p.cb, S, nbk, (const uint32_t*)pos_s, ids, ekeys);
        HG_TRY(hipGetLastError());
    }
    if (p.big_buckets) {
        hipLaunchKernelGGL(k_big_offsets, dim3(grid_of(p.big_buckets)), dim3(kT), 0, s, set_off,
                           bb, (const uint64_t*)p.cb, (const uint64_t*)p.cv, S, p.big_buckets,
                           (const uint32_t*)gb_s, offsets);
        HG_TRY(hipGetLastError());
    }
    uint32_t h_bad = 0;
    HG_TRY(copy_to_host(&h_bad, bad, 4, s));
    HG_TRY(hipStreamSynchronize(s));
    *bad_out = h_bad != 0;
    return hipSuccess;
}

struct PairWs {
    uint32_t *work, *bad;
    uint64_t* W;
    void* sws;
};

size_t layout_pairs(void* base, uint64_t Q, PairWs* w) {
    Carver c(base);
    w->work = c.take<uint32_t>(Q + 1);
    w->W = c.take<uint64_t>(Q + 2);
    w->bad = c.take<uint32_t>(64);
    w->sws = c.take<unsigned char>(scan_ws_bytes(Q + 1));
    return c.off;
}

size_t coll_pairs_ws_bytes(uint64_t Q) {
    PairWs w;
    return layout_pairs(nullptr, Q, &w);
}

template <typename Key>
hipError_t run_coll_intersect(const CollDev& A, const CollDev& B, uint64_t seed,
                              const uint32_t* pairs, uint64_t Q, unsigned long long* counts,
                              uint64_t* h_total, void* ws, bool* bad_out, hipStream_t s) {
    const SetsView a{A.set_off, A.bb, A.offsets, A.keys, A.S};
    const SetsView b{B.set_off, B.bb, B.offsets, B.keys, B.S};
    PairWs pw;
    layout_pairs(ws, Q, &pw);
    uint32_t *work = pw.work, *bad = pw.bad;
    uint64_t* W = pw.W;
    void* sws = pw.sws;
    *bad_out = false;
    HG_TRY(fill_u32(bad, 1, 0u, s));
    if (counts && Q) {
        hipLaunchKernelGGL(k_zero_u64, dim3(grid_of(Q)), dim3(kT), 0, s, counts, Q);
        HG_TRY(hipGetLastError());
    }
    {
        HG_PROF("coll_pair_work", s);
        hipLaunchKernelGGL(k_pair_work, dim3(grid_of(Q + 1)), dim3(kT), 0, s, pairs, Q, a, b, work,
                           bad);
        HG_TRY(hipGetLastError());
        HG_TRY(scan_excl<uint64_t>(work, Q + 1, W, nullptr, sws, s));
    }
    uint64_t T = 0;
    uint32_t h_bad = 0;
    HG_TRY(copy_to_host(&T, W + Q + 1, 8, s));
    HG_TRY(copy_to_host(&h_bad, bad, 4, s));
    HG_TRY(hipStreamSynchronize(s));
    if (h_bad) {
        *bad_out = true;
        return hipSuccess;
    }
    const uint64_t chunks = ceil_div(T, kPairChunk);
    Workspace part(s);
    if (chunks) {
        HG_TRY(part.get((chunks + 1) * sizeof(unsigned long long)));
        HG_PROF("coll_pair_count", s);
        hipLaunchKernelGGL(k_pair_count<Key>, dim3((uint32_t)chunks), dim3(kT), 0, s, pairs,
                           (const uint64_t*)W, Q, T, a, b, seed, counts,
                           (unsigned long long*)part.p);
        HG_TRY(hipGetLastError());
    }
    if (h_total) {
        *h_total = 0;
        if (chunks) {
            unsigned long long* sum = (unsigned long long*)part.p + chunks;
            hipLaunchKernelGGL(k_sum_u64, dim3(1), dim3(1024), 0, s,
                               (const unsigned long long*)part.p, chunks, sum);
            HG_TRY(hipGetLastError());
            HG_TRY(copy_to_host(h_total, sum, 8, s));
            HG_TRY(hipStreamSynchronize(s));
        }
    }
    return hipSuccess;
}

#define HG_COLL_INST(Key)                                                                         \
    template hipError_t run_coll_build<Key>(const Key*, const uint32_t*, uint32_t, uint64_t,      \
                                            const uint64_t*, const CollPlan&, void*, uint32_t*,   \
                                            uint32_t*, Key*, bool*, hipStream_t);                 \
    template hipError_t run_coll_intersect<Key>(const CollDev&, const CollDev&, uint64_t,         \
                                                const uint32_t*, uint64_t, unsigned long long*,   \
                                                uint64_t*, void*, bool*, hipStream_t);
HG_COLL_INST(uint32_t)
HG_COLL_INST(uint64_t)
#undef HG_COLL_INST

}  // namespace hg
