// Key-run summaries of long buckets: exact probing under skew.
//
// Probe-Standard (Sec. 3.4) scans a query's whole bucket.  When many entries
// share a bucket -- heavy duplication, or Zipf keys where one key holds a
// large share of the input -- every probe of that bucket pays its full
// length, so a skewed join costs as much as the number of matching pairs.
// For each bucket longer than kRunBucket the table therefore also keeps the
// bucket's distinct keys in ascending order (its runs), each with the end of
// its group in `kperm`, a copy of the bucket's ids grouped by key (bucket
// order inside each group).  A probe of a long bucket binary-searches the
// runs; its pairs are the ids of one group.  Counts and pairs are exactly
// those of a scan.  The arrays are parallel to the edge array (see RunsDev),
// so every bucket's summary has a fixed place and nothing is sized on the
// host: a build with the index never waits for the device.
//
// Most long buckets are built inside the per-bin kernel, from LDS
// (bin_long_runs): a long bucket is usually one key repeated (duplicates) or
// dominated by one key (skew), so the entries equal to the bucket's first key
// (the lead key) form one run and the few others are sorted across a wave.
// This file holds the general pass for the rest, which the per-bin kernels
// list per bin:
//   * buckets of up to light_cap keys (one workgroup each, in LDS): the
//     others are gathered, sorted (bitonic network in LDS) and cut into runs;
//   * longer buckets (from bins too large for LDS), in chunks of kChunk
//     entries spread over the grid: per chunk the others and those below the
//     lead key are counted, a per-bucket scan turns the counts into chunk
//     bases, each chunk then writes its others contiguously to scratch and its
//     lead ids to kperm, and one workgroup per bucket sorts the others (LDS,
//     or a workgroup-wide radix sort through global memory when they exceed
//     LDS) and writes their runs.
// Every kernel takes its amount of work from device counters and strides
// over it with a fixed grid.
#include "hg_v2_device.h"

namespace hg {

namespace {

using namespace v2dev;

constexpr int kRT = kLocalThreads;      // threads of the per-bucket kernels (512)
constexpr int kCT = 256;                // threads of the per-chunk kernels
constexpr int kCItems = 16;             // consecutive entries per thread of a chunk
constexpr uint32_t kChunk = kCT * kCItems;  // 4096
constexpr uint32_t kGenGrid = 2048;
constexpr uint32_t kChunkGrid = 2048;
constexpr uint32_t kBucketGrid = 512;

// Entries the LDS sort of a bucket's other keys holds: light_cap rounded up
// to a power of two (8192 for 32-bit keys, 4096 for 64-bit keys).
template <typename Key>
constexpr uint32_t lds_sort_cap() {
    return sizeof(Key) == 8 ? 4096u : 8192u;
}

// Buckets longer than light_cap go through the chunked path.
template <typename Key>
constexpr uint32_t small_cap() {
    return light_cap<Key>();
}

template <typename Key>
__device__ __forceinline__ uint32_t key32(Key k) {
    return sizeof(Key) == 4 ? (uint32_t)k : 0u;
}

// LDS of the per-bucket kernels: sort buffer, radix counters, scan temporaries.
template <typename Key>
struct BucketLds {
    Key* sk;          // [lds_sort_cap]
    uint32_t* sp;     // [lds_sort_cap]
    uint32_t* wcnt;   // [W_LOCAL * 256]
    uint32_t* dstart; // [256]
    uint32_t* base;   // [256]
    uint32_t* tmp;    // [2 * W_LOCAL + 2]
    uint32_t* sh;     // [8] broadcast words
    __host__ __device__ static constexpr size_t bytes() {
        return (size_t)lds_sort_cap<Key>() * (sizeof(Key) + 4) + 4 * (W_LOCAL * 256 + 256 + 256 +
                                                                     2 * W_LOCAL + 2 + 8) + 64;
    }
    __device__ explicit BucketLds(unsigned char* p) {
        sk = (Key*)p;
        sp = (uint32_t*)(sk + lds_sort_cap<Key>());
        wcnt = sp + lds_sort_cap<Key>();
        dstart = wcnt + W_LOCAL * 256;
        base = dstart + 256;
        tmp = base + 256;
        sh = tmp + 2 * W_LOCAL + 2;
    }
};

// Bitonic sort of n2 (a power of two) (key, position) pairs in LDS,
// ascending; positions are distinct, so the order is total.  Barriers.
template <typename Key>
__device__ void lds_bitonic(Key* k, uint32_t* p, uint32_t n2) {
    for (uint32_t size = 2; size <= n2; size <<= 1)
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < n2 / 2; i += kRT) {
                const uint32_t lo = 2 * stride * (i / stride) + (i % stride), hi = lo + stride;
                const bool up = (lo & size) == 0;
                const Key ka = k[lo], kb = k[hi];
                const uint32_t pa = p[lo], pb = p[hi];
                const bool b_less = kb < ka || (kb == ka && pb < pa);
                if (b_less == up) {
                    k[lo] = kb;
                    k[hi] = ka;
                    p[lo] = pb;
                    p[hi] = pa;
                }
            }
            __syncthreads();
        }
}

// Stable LSD radix sort (8-bit digits, every bit of the key) of O pairs
// through global memory by one workgroup: (ka, pa) -> (kb, pb) -> ... The
// number of passes is even, so the result ends in (ka, pa).  Barriers.
template <typename Key>
__device__ void wg_radix_sort(Key* ka, uint32_t* pa, Key* kb, uint32_t* pb, uint32_t O,
                              const BucketLds<Key>& m) {
    constexpr int IT = 8;
    constexpr uint32_t tile = kRT * IT;
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    for (uint32_t shift = 0; shift < sizeof(Key) * 8; shift += 8) {
        for (uint32_t d = threadIdx.x; d < 256; d += kRT) m.base[d] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < O; i += kRT)
            atomicAdd(&m.base[(uint32_t)(ka[i] >> shift) & 255u], 1u);
        __syncthreads();
        uint32_t all;
        const uint32_t v = threadIdx.x < 256 ? m.base[threadIdx.x] : 0u;
        const uint32_t ex = block_excl_scan<kRT>(v, m.tmp, &all);
        if (threadIdx.x < 256) m.base[threadIdx.x] = ex;
        __syncthreads();
        for (uint32_t t0 = 0; t0 < O; t0 += tile) {
            const uint32_t cnt = O - t0 < tile ? O - t0 : tile;
            Key k[IT];
            uint32_t p[IT], dig[IT], pos[IT];
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                const uint32_t e = w * (kWave * IT) + r * kWave + lane;
                if (e < cnt) {
                    k[r] = ka[t0 + e];
                    p[r] = pa[t0 + e];
                    dig[r] = (uint32_t)(k[r] >> shift) & 255u;
                } else {
                    k[r] = 0;
                    p[r] = 0;
                    dig[r] = 256u;  // ignored by the ranking
                }
            }
            rank_stable<kRT, IT>(dig, 8, m.wcnt, m.dstart, m.tmp, pos);
#pragma unroll
            for (int r = 0; r < IT; ++r)
                if (dig[r] < 256u) {
                    const uint32_t o = m.base[dig[r]] + pos[r] - m.dstart[dig[r]];
                    kb[o] = k[r];
                    pb[o] = p[r];
                }
            __syncthreads();
            for (uint32_t d = threadIdx.x; d < 256; d += kRT)
                m.base[d] += (d + 1 < 256 ? m.dstart[d + 1] : cnt) - m.dstart[d];
            __syncthreads();
        }
        Key* tk = ka;
        ka = kb;
        kb = tk;
        uint32_t* tp = pa;
        pa = pb;
        pb = tp;
    }
}

// Runs of a long bucket (edge positions [st, st + len), lead key `lead`) from
// its O > 0 other entries sorted by (key, position in the bucket) in sk / sp:
// every other entry's id goes to kperm (before the lead key's group when its
// key is smaller, after it otherwise), every run gets its key and end, the
// lead run is slotted in, and the bucket's index entry points at the runs.
// The lead key's ids are written by the caller.  Returns (via m.sh[0]) the
// number of others below the lead key.  Whole workgroup; barriers.
template <typename Key>
__device__ void emit_runs(const Key* sk, const uint32_t* sp, uint32_t O, Key lead, uint32_t len,
                          uint32_t st, uint32_t b, const uint32_t* __restrict__ ids,
                          const IndexOut& ix, const BucketLds<Key>& m) {
    Key* rkey = (Key*)ix.runs.run_key;
    uint32_t* rend = ix.runs.run_end;
    uint32_t* kperm = ix.runs.kperm;
    if (threadIdx.x == 0) {
        uint32_t lo = 0, hi = O;  // others below the lead key
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (sk[mid] < lead) lo = mid + 1;
            else hi = mid;
        }
        m.sh[0] = lo;
        m.sh[1] = 0;  // runs below the lead key
    }
    __syncthreads();
    const uint32_t nless = m.sh[0], clead = len - O;
    uint32_t runs = 0;  // other runs before this tile
    for (uint32_t t0 = 0; t0 < O; t0 += kRT) {
        const uint32_t i = t0 + threadIdx.x;
        const bool valid = i < O;
        const Key k = valid ? sk[i] : (Key)0;
        const bool first = valid && (i == 0 || sk[i - 1] != k);
        const bool last = valid && (i + 1 == O || sk[i + 1] != k);
        uint32_t all;
        const uint32_t ex = block_excl_scan<kRT>(first ? 1u : 0u, m.tmp, &all);
        if (valid) {
            const bool below = i < nless;
            const uint32_t ro = runs + ex + (first ? 1u : 0u) - 1u;  // run among the others
            const uint32_t r = ro + (below ? 0u : 1u);
            kperm[st + i + (below ? 0u : clead)] = ids[st + sp[i]];
            if (first) rkey[st + r] = k;
            if (last) rend[st + r] = i + 1 + (below ? 0u : clead);
            if (i + 1 == nless) m.sh[1] = ro + 1;
        }
        runs += all;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t rl = m.sh[1];
        rkey[st + rl] = lead;
        rend[st + rl] = nless + clead;
        ix.head[b] = make_uint4(len, st, runs + 1, 0u);
    }
    __syncthreads();
}

// A bucket of one key: a single run, no kperm (its ids are the edge array's).
template <typename Key>
__device__ __forceinline__ void single_run(const IndexOut& ix, uint32_t b, uint32_t st,
                                           uint32_t len, Key lead) {
    ((Key*)ix.runs.run_key)[st] = lead;
    ix.runs.run_end[st] = len;
    ix.head[b] = make_uint4(len, st, 1u, key32(lead));
}

struct G2 {
    uint32_t* list;    // [cap] bucket ids
    uint32_t* c0;      // [cap] first chunk
    uint32_t* info;    // [2 * cap] others, others below the lead key
    uint32_t* owner;   // [chunks] bucket (index in list) of each chunk
    uint32_t* oth;     // [chunks] others, then their exclusive prefix in the bucket
    uint32_t* less;    // [chunks] others below the lead key, then their prefix
    uint32_t cap, chunk_cap;
};

struct G2Layout {
    G2 g;
    size_t bytes;
};

G2Layout layout_g2(void* ws, uint64_t n) {
    Carver c(ws);
    G2 g{};
    g.cap = (uint32_t)(n / (light_cap<uint64_t>() + 1) + 1);
    g.chunk_cap = (uint32_t)(n / kChunk + g.cap + 1);
    g.list = c.take<uint32_t>(g.cap);
    g.c0 = c.take<uint32_t>(g.cap);
    g.info = c.take<uint32_t>(2 * (size_t)g.cap);
    g.owner = c.take<uint32_t>(g.chunk_cap);
    g.oth = c.take<uint32_t>(g.chunk_cap);
    g.less = c.take<uint32_t>(g.chunk_cap);
    return G2Layout{g, c.off + 256};
}

// The listed long buckets of every bin: first each wave finishes the buckets
// whose entries other than the lead key fit its lanes (marking them done in
// the list), then the workgroup sorts the other small ones in LDS; longer ones
// are handed to the chunked path (ctr[0] buckets, ctr[1] chunks).
template <typename Key>
__global__ __launch_bounds__(kRT) void k_runs_general(
    const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ ids,
    const Key* __restrict__ ekeys, const uint32_t* __restrict__ bin_start, uint32_t bins,
    IndexOut ix, G2 g2, uint32_t* __restrict__ ctr) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BucketLds<Key> m(smem);
    for (uint32_t g = blockIdx.x; g < bins; g += gridDim.x) {
        const uint32_t listed = ix.gen_cnt[g];
        if (listed == 0) continue;  // uniform across the workgroup
        uint32_t* list = ix.gen_list + gen_region(bin_start[g], g);
        {
            // a wave per bucket, its 64-entry buffers in the sort buffers
            const uint32_t w = threadIdx.x / kWave, lane = lane_id();
            Key* bk = m.sk + w * kWave;
            uint16_t* bp = (uint16_t*)m.sp + w * kWave;
            for (uint32_t t = w; t < listed; t += W_LOCAL) {
                const uint32_t b = list[t];
                const uint32_t st = offsets[b], len = offsets[b + 1] - st;
                // (a bucket much longer than a wave rarely has its other
                // keys fit one; it goes to the workgroup below directly)
                if (len > 4u * kWave) continue;
                if (wave_bucket_runs<Key>(ix, ekeys, ids, st, st + len, st, b, bk, bp) &&
                    lane == 0)
                    list[t] = ~0u;  // done
            }
        }
        __syncthreads();
        for (uint32_t t = 0; t < listed; ++t) {
            const uint32_t b = list[t];
            if (b == ~0u) continue;  // uniform: finished by a wave above
            const uint32_t st = offsets[b], len = offsets[b + 1] - st;
            const Key lead = ekeys[st];
            if (len > small_cap<Key>()) {
                if (threadIdx.x == 0) {
                    const uint32_t nch = (len + kChunk - 1) / kChunk;
                    const uint32_t i = atomicAdd(&ctr[0], 1u);
                    const uint32_t c0 = atomicAdd(&ctr[1], nch);
                    m.sh[2] = i;
                    m.sh[3] = c0;
                    if (i < g2.cap && c0 + nch <= g2.chunk_cap) {
                        g2.list[i] = b;
                        g2.c0[i] = c0;
                    }
                }
                __syncthreads();
                const uint32_t i = m.sh[2], c0 = m.sh[3];
                const uint32_t nch = (len + kChunk - 1) / kChunk;
                if (i < g2.cap && c0 + nch <= g2.chunk_cap)
                    for (uint32_t j = threadIdx.x; j < nch; j += kRT) g2.owner[c0 + j] = i;
                __syncthreads();
                continue;
            }
            // gather the entries that differ from the lead key, in bucket order
            uint32_t O = 0;
            for (uint32_t c = 0; c < len; c += kRT) {
                const uint32_t i = c + threadIdx.x;
                const Key x = i < len ? ekeys[st + i] : lead;
                const bool o = x != lead;
                uint32_t all;
                const uint32_t ex = block_excl_scan<kRT>(o ? 1u : 0u, m.tmp, &all);
                if (o) {
                    m.sk[O + ex] = x;
                    m.sp[O + ex] = i;
                }
                O += all;
            }
            if (O == 0) {
                if (threadIdx.x == 0) single_run<Key>(ix, b, st, len, lead);
                __syncthreads();
                continue;
            }
            uint32_t n2 = 1;
            while (n2 < O) n2 <<= 1;
            for (uint32_t i = O + threadIdx.x; i < n2; i += kRT) {
                m.sk[i] = (Key)~(Key)0;
                m.sp[i] = 0xffffffffu;
            }
            __syncthreads();
            lds_bitonic<Key>(m.sk, m.sp, n2);
            emit_runs<Key>(m.sk, m.sp, O, lead, len, st, b, ids, ix, m);
            // the lead key's ids, in bucket order, after the smaller keys
            const uint32_t nless = m.sh[0];
            uint32_t done = 0;
            for (uint32_t c = 0; c < len; c += kRT) {
                const uint32_t i = c + threadIdx.x;
                const bool isl = i < len && ekeys[st + i] == lead;
                uint32_t all;
                const uint32_t ex = block_excl_scan<kRT>(isl ? 1u : 0u, m.tmp, &all);
                if (isl) ix.runs.kperm[st + nless + done + ex] = ids[st + i];
                done += all;
            }
            __syncthreads();
        }
    }
}

// Chunk c of a long bucket: thread t holds entries [t*16, t*16 + 16) of the
// chunk (consecutive, so thread order is bucket order).
struct ChunkRef {
    uint32_t i, b, st, len, base, cl;
};

template <typename Key>
__device__ __forceinline__ ChunkRef chunk_at(uint32_t c, const G2& g2,
                                             const uint32_t* __restrict__ offsets) {
    ChunkRef r;
    r.i = g2.owner[c];
    r.b = g2.list[r.i];
    r.st = offsets[r.b];
    r.len = offsets[r.b + 1] - r.st;
    r.base = (c - g2.c0[r.i]) * kChunk;
    r.cl = r.len - r.base < kChunk ? r.len - r.base : kChunk;
    return r;
}

// Per chunk: entries that differ from the lead key, and of them those below it.
template <typename Key>
__global__ __launch_bounds__(kCT) void k_runs_chunk_count(const uint32_t* __restrict__ offsets,
                                                          const Key* __restrict__ ekeys, G2 g2,
                                                          const uint32_t* __restrict__ ctr) {
    __shared__ uint32_t red[2 * (kCT / kWave)];
    const uint32_t nch = ctr[1] < g2.chunk_cap ? ctr[1] : g2.chunk_cap;
    for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const ChunkRef r = chunk_at<Key>(c, g2, offsets);
        const Key lead = ekeys[r.st];
        uint32_t o = 0, l = 0;
#pragma unroll 4
        for (int j = 0; j < kCItems; ++j) {
            const uint32_t e = threadIdx.x * kCItems + j;
            if (e < r.cl) {
                const Key x = ekeys[r.st + r.base + e];
                o += x != lead;
                l += x < lead;
            }
        }
        o = wave_sum(o);
        l = wave_sum(l);
        if (lane_id() == 0) {
            red[threadIdx.x / kWave] = o;
            red[kCT / kWave + threadIdx.x / kWave] = l;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t so = 0, sl = 0;
            for (int q = 0; q < kCT / kWave; ++q) {
                so += red[q];
                sl += red[kCT / kWave + q];
            }
            g2.oth[c] = so;
            g2.less[c] = sl;
        }
        __syncthreads();
    }
}

// Per long bucket: exclusive prefixes of its chunks' counts (in place), the
// totals, and a bucket of one key finished outright.
template <typename Key>
__global__ __launch_bounds__(kRT) void k_runs_chunk_scan(const uint32_t* __restrict__ offsets,
                                                         const Key* __restrict__ ekeys,
                                                         IndexOut ix, G2 g2,
                                                         const uint32_t* __restrict__ ctr) {
    __shared__ uint32_t tmp[kRT / kWave + 1];
    const uint32_t nb2 = ctr[0] < g2.cap ? ctr[0] : g2.cap;
    for (uint32_t i = blockIdx.x; i < nb2; i += gridDim.x) {
        const uint32_t b = g2.list[i], c0 = g2.c0[i];
        const uint32_t st = offsets[b], len = offsets[b + 1] - st;
        const uint32_t nch = (len + kChunk - 1) / kChunk;
        uint32_t co = 0, cl = 0;
        for (uint32_t t0 = 0; t0 < nch; t0 += kRT) {
            const uint32_t j = t0 + threadIdx.x;
            const uint32_t vo = j < nch ? g2.oth[c0 + j] : 0u;
            const uint32_t vl = j < nch ? g2.less[c0 + j] : 0u;
            uint32_t ao, al;
            const uint32_t eo = block_excl_scan<kRT>(vo, tmp, &ao);
            const uint32_t el = block_excl_scan<kRT>(vl, tmp, &al);
            if (j < nch) {
                g2.oth[c0 + j] = co + eo;
                g2.less[c0 + j] = cl + el;
            }
            co += ao;
            cl += al;
        }
        if (threadIdx.x == 0) {
            g2.info[2 * i] = co;
            g2.info[2 * i + 1] = cl;
            if (co == 0) single_run<Key>(ix, b, st, len, ekeys[st]);
        }
    }
}

// Per chunk (buckets with other keys): the others go contiguously to the
// scratch arrays (key, position in the bucket), the lead key's ids to kperm
// after the smaller keys' groups.
template <typename Key>
__global__ __launch_bounds__(kCT) void k_runs_chunk_scatter(
    const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ ids,
    const Key* __restrict__ ekeys, IndexOut ix, G2 g2, const uint32_t* __restrict__ ctr,
    Key* __restrict__ skey, uint32_t* __restrict__ spos) {
    __shared__ uint32_t tmp[kCT / kWave + 1];
    const uint32_t nch = ctr[1] < g2.chunk_cap ? ctr[1] : g2.chunk_cap;
    for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const ChunkRef r = chunk_at<Key>(c, g2, offsets);
        const uint32_t O = g2.info[2 * r.i], nless = g2.info[2 * r.i + 1];
        if (O == 0) continue;  // uniform: a single run, no kperm
        const Key lead = ekeys[r.st];
        const uint32_t obase = g2.oth[c], lbase = r.base - obase;
        Key x[kCItems];
        uint32_t mine = 0;
#pragma unroll
        for (int j = 0; j < kCItems; ++j) {
            const uint32_t e = threadIdx.x * kCItems + j;
            x[j] = e < r.cl ? ekeys[r.st + r.base + e] : lead;
            mine += x[j] != lead;
        }
        uint32_t all;
        uint32_t o = obase + block_excl_scan<kCT>(mine, tmp, &all);
        uint32_t l = lbase + threadIdx.x * kCItems - (o - obase);
#pragma unroll
        for (int j = 0; j < kCItems; ++j) {
            // a predicate rather than a break, so that the loop unrolls and
            // x[] stays in registers
            const uint32_t e = threadIdx.x * kCItems + j;
            if (e < r.cl) {
                if (x[j] != lead) {
                    skey[r.st + o] = x[j];
                    spos[r.st + o] = r.base + e;
                    ++o;
                } else {
                    ix.runs.kperm[r.st + nless + l] = ids[r.st + r.base + e];
                    ++l;
                }
            }
        }
    }
}

// Per long bucket with other keys: sort the others (LDS when they fit, else a
// workgroup radix sort through global memory) and write their runs.
template <typename Key>
__global__ __launch_bounds__(kRT) void k_runs_chunk_sort(
    const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ ids,
    const Key* __restrict__ ekeys, IndexOut ix, G2 g2, const uint32_t* __restrict__ ctr,
    Key* __restrict__ skey, uint32_t* __restrict__ spos) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BucketLds<Key> m(smem);
    const uint32_t nb2 = ctr[0] < g2.cap ? ctr[0] : g2.cap;
    for (uint32_t i = blockIdx.x; i < nb2; i += gridDim.x) {
        const uint32_t O = g2.info[2 * i];
        if (O == 0) continue;
        const uint32_t b = g2.list[i];
        const uint32_t st = offsets[b], len = offsets[b + 1] - st;
        const Key lead = ekeys[st];
        if (O <= lds_sort_cap<Key>()) {
            uint32_t n2 = 1;
            while (n2 < O) n2 <<= 1;
            for (uint32_t t = threadIdx.x; t < n2; t += kRT) {
                m.sk[t] = t < O ? skey[st + t] : (Key)~(Key)0;
                m.sp[t] = t < O ? spos[st + t] : 0xffffffffu;
            }
            __syncthreads();
            lds_bitonic<Key>(m.sk, m.sp, n2);
            emit_runs<Key>(m.sk, m.sp, O, lead, len, st, b, ids, ix, m);
        } else {
            // the run arrays of [st, st + O) serve as the second buffer; the
            // sorted pairs end back in the scratch arrays
            wg_radix_sort<Key>(skey + st, spos + st, (Key*)ix.runs.run_key + st,
                               ix.runs.run_end + st, O, m);
            emit_runs<Key>(skey + st, spos + st, O, lead, len, st, b, ids, ix, m);
        }
    }
}

template <typename Key>
hipError_t set_runs_smem() {
    static std::atomic<uint64_t> done{0};
    return once_per_device(done, [] {
        const int lim = 160 * 1024;
        HG_TRY(hipFuncSetAttribute((const void*)k_runs_general<Key>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_runs_chunk_sort<Key>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        return hipSuccess;
    });
}

}  // namespace

size_t runs_ws_bytes(uint64_t n, uint64_t bins) {
    (void)bins;
    return layout_g2(nullptr, n).bytes;
}

template <typename Key>
hipError_t run_key_runs(const uint32_t* offsets, const uint32_t* ids, const Key* ekeys,
                        uint64_t n, const uint32_t* bin_start, uint32_t bins, const IndexOut& ix,
                        Key* rkeys, uint32_t* rids, uint32_t* ctr, void* ws, hipStream_t s) {
    if (n == 0 || bins == 0) return hipSuccess;
    HG_TRY(set_runs_smem<Key>());
    const G2 g2 = layout_g2(ws, n).g;
    const size_t lds = BucketLds<Key>::bytes();
    HG_PROF("runs_build", s);
    const uint32_t gg = bins < kGenGrid ? bins : kGenGrid;
    hipLaunchKernelGGL(k_runs_general<Key>, dim3(gg), dim3(kRT), lds, s, offsets, ids, ekeys,
                       bin_start, bins, ix, g2, ctr);
    HG_TRY(hipGetLastError());
    // the chunked path: grids sized for the most work there can be, strided
    // over what the counters hold
    const uint32_t cg = (uint32_t)(g2.chunk_cap < kChunkGrid ? g2.chunk_cap : kChunkGrid);
    const uint32_t bg = g2.cap < kBucketGrid ? g2.cap : kBucketGrid;
    hipLaunchKernelGGL(k_runs_chunk_count<Key>, dim3(cg), dim3(kCT), 0, s, offsets, ekeys, g2,
                       (const uint32_t*)ctr);
    HG_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_runs_chunk_scan<Key>, dim3(bg), dim3(kRT), 0, s, offsets, ekeys, ix, g2,
                       (const uint32_t*)ctr);
    HG_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_runs_chunk_scatter<Key>, dim3(cg), dim3(kCT), 0, s, offsets, ids, ekeys,
                       ix, g2, (const uint32_t*)ctr, rkeys, rids);
    HG_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_runs_chunk_sort<Key>, dim3(bg), dim3(kRT), lds, s, offsets, ids, ekeys, ix,
                       g2, (const uint32_t*)ctr, rkeys, rids);
    return hipGetLastError();
}

template hipError_t run_key_runs<uint32_t>(const uint32_t*, const uint32_t*, const uint32_t*,
                                           uint64_t, const uint32_t*, uint32_t, const IndexOut&,
                                           uint32_t*, uint32_t*, uint32_t*, void*, hipStream_t);
template hipError_t run_key_runs<uint64_t>(const uint32_t*, const uint32_t*, const uint64_t*,
                                           uint64_t, const uint32_t*, uint32_t, const IndexOut&,
                                           uint64_t*, uint32_t*, uint32_t*, void*, hipStream_t);

}  // namespace hg
