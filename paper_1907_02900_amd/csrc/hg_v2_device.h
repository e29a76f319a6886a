// Device code shared by the single-table V2 build (hg_v2.hip) and the batched
// build (hg_batch.hip): stable ranking of a tile by a digit, in-LDS sorting of
// a bin by bucket, and the per-bin build bodies.
#pragma once

#include "hg_internal.h"

namespace hg {
namespace v2dev {

constexpr int W_PART = kPartThreads / kWave;
constexpr int W_LOCAL = kLocalThreads / kWave;
constexpr uint32_t kFixMax = 16;  // longest bucket the insertion-sort path handles

// ------------------------------------------------------------ ranking -----

// Digit-major exclusive scan of the per-wave digit counters wcnt[w][d]
// (W waves, D digits): afterwards wcnt[w][d] holds the position of wave w's
// first item of digit d in the stably sorted tile, and dstart[d] the start
// of digit d.  Barrier on exit.
template <int THREADS>
__device__ __forceinline__ void scan_wave_digit_counts(uint32_t D, uint32_t* wcnt,
                                                       uint32_t* dstart, uint32_t* tmp) {
    constexpr int W = THREADS / kWave;
    const uint32_t per = (D + THREADS - 1) / THREADS;
    const uint32_t d0 = threadIdx.x * per;
    uint32_t mine = 0;
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t d = d0 + j;
        if (d < D)
#pragma unroll
            for (int w = 0; w < W; ++w) mine += wcnt[w * D + d];
    }
    uint32_t all;
    uint32_t run = block_excl_scan<THREADS>(mine, tmp, &all);
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t d = d0 + j;
        if (d < D) {
            dstart[d] = run;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint32_t v = wcnt[w * D + d];
                wcnt[w * D + d] = run;
                run += v;
            }
        }
    }
    __syncthreads();
}

// Stable rank of up to 64*ITEMS items per wave by a digit of `bits` bits
// (D = 2^bits <= 2048).  Item r of a lane is entry (wave base + r*64 + lane);
// items with dig >= D are ignored.  Per round every lane reads its digit's
// running count in the wave's counter row and the lowest lane of each group
// of equal digits adds the group's size with a non-returning LDS atomic.  LDS
// performs a wave's operations in issue order, so a read sees exactly the
// items of the wave's earlier rounds, and no round waits for the previous
// one.  Every round runs unconditionally (a round without valid items costs
// its ballots and changes nothing), which keeps the code straight-line.  On
// return pos[r] is the item's index in the tile sorted stably by digit
// (undefined for ignored items).  Contains barriers.
template <int THREADS, int ITEMS>
__device__ __forceinline__ void rank_stable(const uint32_t (&dig)[ITEMS], uint32_t bits,
                                            uint32_t* wcnt, uint32_t* dstart, uint32_t* tmp,
                                            uint32_t (&pos)[ITEMS]) {
    constexpr int W = THREADS / kWave;
    const uint32_t D = 1u << bits, mask = D - 1;
    const uint32_t w = threadIdx.x / kWave;
    for (uint32_t i = threadIdx.x; i < W * D; i += THREADS) wcnt[i] = 0;
    __syncthreads();
    uint32_t* my = wcnt + w * D;
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t d = dig[r];
        const bool valid = d < D;
        const uint64_t peers = match_digit(d, (int)bits, ballot(valid));
        const uint32_t below = mbcnt(peers);
        pos[r] = my[d & mask] + below;
        if (valid && below == 0)
            __hip_atomic_fetch_add(&my[d], (uint32_t)__popcll(peers), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    scan_wave_digit_counts<THREADS>(D, wcnt, dstart, tmp);
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) pos[r] += my[dig[r] & mask];
}

// Rank of up to THREADS*ITEMS items by a digit of `bits` bits with no order
// among equal digits: one returning LDS atomic per item on per-workgroup
// counters, then an exclusive scan of the counts.  pos[r] is the item's index
// in the tile grouped by digit (undefined for items with dig >= D);
// dstart[d] the start of digit d.  `cnt` holds D counters.  Contains
// barriers.
template <int THREADS, int ITEMS>
__device__ __forceinline__ void rank_any(const uint32_t (&dig)[ITEMS], uint32_t bits,
                                         uint32_t* cnt, uint32_t* dstart, uint32_t* tmp,
                                         uint32_t (&pos)[ITEMS]) {
    const uint32_t D = 1u << bits, mask = D - 1;
    for (uint32_t i = threadIdx.x; i < D; i += THREADS) cnt[i] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
        if (dig[r] < D) pos[r] = atomicAdd(&cnt[dig[r]], 1u);
    __syncthreads();
    const uint32_t per = (D + THREADS - 1) / THREADS;
    const uint32_t d0 = threadIdx.x * per;
    uint32_t mine = 0;
    for (uint32_t j = 0; j < per; ++j)
        if (d0 + j < D) mine += cnt[d0 + j];
    uint32_t all;
    uint32_t run = block_excl_scan<THREADS>(mine, tmp, &all);
    for (uint32_t j = 0; j < per; ++j)
        if (d0 + j < D) {
            dstart[d0 + j] = run;
            run += cnt[d0 + j];
        }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) pos[r] += dstart[dig[r] & mask];
}

// -------------------------------------------------- per-bin LDS build -----

// Place one chunk of <= ITEMS*64*W entries held in registers: two stable LSD
// ranking passes over the local bucket index (lo bits, then hi bits) leave
// the chunk sorted by bucket in skeys/sids/sb.  Items are balanced over the
// waves: wave w owns entries [w*chunk, (w+1)*chunk).
template <typename Key, int ITEMS>
__device__ __forceinline__ void sort_chunk_by_bucket(Key (&kk)[ITEMS], uint32_t (&id)[ITEMS],
                                                     uint32_t (&b)[ITEMS], uint32_t rounds,
                                                     uint32_t cl, uint32_t wchunk, uint32_t k,
                                                     Key* skeys, uint32_t* sids, uint16_t* sb,
                                                     uint32_t* wcnt, uint32_t* dstart,
                                                     uint32_t* tmp) {
    const uint32_t NB = 1u << k;
    const uint32_t lo_bits = (k + 1) / 2, hi_bits = k / 2;
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    uint32_t dig[ITEMS], pos[ITEMS];
    if (k == 0) {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const uint32_t e = w * wchunk + r * kWave + lane;
            if ((uint32_t)r < rounds && r * kWave + lane < wchunk && e < cl) {
                skeys[e] = kk[r];
                sids[e] = id[r];
                sb[e] = 0;
            }
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) dig[r] = (b[r] < NB) ? (b[r] & ((1u << lo_bits) - 1)) : 64u;
    rank_stable<kLocalThreads, ITEMS>(dig, lo_bits, wcnt, dstart, tmp, pos);
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
        if ((uint32_t)r < rounds && b[r] < NB) {
            skeys[pos[r]] = kk[r];
            sids[pos[r]] = id[r];
            sb[pos[r]] = (uint16_t)b[r];
        }
    __syncthreads();
    if (hi_bits == 0) return;
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t e = w * wchunk + r * kWave + lane;
        if ((uint32_t)r < rounds && r * kWave + lane < wchunk && e < cl) {
            kk[r] = skeys[e];
            id[r] = sids[e];
            b[r] = sb[e];
            dig[r] = b[r] >> lo_bits;
        } else {
            b[r] = NB;
            dig[r] = 64u;
        }
    }
    // rank_stable synchronises before counting, so every wave has finished
    // reading the buffers before any wave overwrites them below
    rank_stable<kLocalThreads, ITEMS>(dig, hi_bits, wcnt, dstart, tmp, pos);
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
        if ((uint32_t)r < rounds && b[r] < NB) {
            skeys[pos[r]] = kk[r];
            sids[pos[r]] = id[r];
            sb[pos[r]] = (uint16_t)b[r];
        }
}

// Put the s <= 8 entries of one bucket in LDS (ids[0..s), keys[0..s)) in
// ascending id order, in registers: load them, run Batcher's odd-even merge
// network for 8 (19 compare-exchanges; empty places hold id 0xffffffff,
// above every real id, and sort last), store them back.  Unlike an insertion
// sort in LDS it has no chain of dependent LDS reads.
template <typename Key>
__device__ __forceinline__ void sort8_by_id(uint32_t* ids, Key* keys, uint32_t s) {
    uint32_t a[8];
    Key k[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = (uint32_t)j < s ? ids[j] : 0xffffffffu;
        k[j] = (uint32_t)j < s ? keys[j] : Key(0);
    }
    auto cx = [&](int i, int j) {
        const bool sw = a[j] < a[i];
        const uint32_t ai = sw ? a[j] : a[i], aj = sw ? a[i] : a[j];
        const Key ki = sw ? k[j] : k[i], kj = sw ? k[i] : k[j];
        a[i] = ai;
        a[j] = aj;
        k[i] = ki;
        k[j] = kj;
    };
    cx(0, 1); cx(2, 3); cx(4, 5); cx(6, 7);
    cx(0, 2); cx(1, 3); cx(4, 6); cx(5, 7);
    cx(1, 2); cx(5, 6);
    cx(0, 4); cx(1, 5); cx(2, 6); cx(3, 7);
    cx(2, 4); cx(3, 5);
    cx(1, 2); cx(3, 4); cx(5, 6);
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if ((uint32_t)j < s) {
            ids[j] = a[j];
            keys[j] = k[j];
        }
}

// Exclusive scan of cnt[0..NB) in place (NB a power of two); returns via
// cnt; *total gets the sum.  All threads must call it.
__device__ __forceinline__ void scan_counts(uint32_t* cnt, uint32_t NB, uint32_t base,
                                            uint32_t* tmp) {
    const uint32_t per = NB >= (uint32_t)kLocalThreads ? NB / kLocalThreads : 1u;
    const uint32_t i0 = threadIdx.x * per;
    uint32_t v[16];
    uint32_t mine = 0;
    for (uint32_t j = 0; j < per; ++j) {
        v[j] = (i0 + j < NB) ? cnt[i0 + j] : 0u;
        mine += v[j];
    }
    uint32_t all;
    uint32_t run = base + block_excl_scan<kLocalThreads>(mine, tmp, &all);
    for (uint32_t j = 0; j < per; ++j)
        if (i0 + j < NB) {
            cnt[i0 + j] = run;
            run += v[j];
        }
    __syncthreads();
}

// Exclusive scan of cnt[0..NB) in place (base 0); returns the largest count.
// `tmp` needs 2 * (waves per block) words.  All threads must call it.
__device__ __forceinline__ uint32_t scan_counts_max(uint32_t* cnt, uint32_t NB, uint32_t* tmp) {
    const uint32_t per = NB >= (uint32_t)kLocalThreads ? NB / kLocalThreads : 1u;
    const uint32_t i0 = threadIdx.x * per;
    uint32_t v[16];
    uint32_t mine = 0, mx = 0;
    for (uint32_t j = 0; j < per; ++j) {
        v[j] = (i0 + j < NB) ? cnt[i0 + j] : 0u;
        mine += v[j];
        mx = v[j] > mx ? v[j] : mx;
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(mx, d, kWave);
        mx = o > mx ? o : mx;
    }
    uint32_t all;
    uint32_t run = block_excl_scan<kLocalThreads>(mine, tmp, &all);
    if (lane_id() == 0) tmp[W_LOCAL + threadIdx.x / kWave] = mx;
    for (uint32_t j = 0; j < per; ++j)
        if (i0 + j < NB) {
            cnt[i0 + j] = run;
            run += v[j];
        }
    __syncthreads();
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < W_LOCAL; ++i) m = tmp[W_LOCAL + i] > m ? tmp[W_LOCAL + i] : m;
    __syncthreads();
    return m;
}

// LDS bytes of light_bin_body / heavy_bin_body for 2^k buckets per bin.
template <typename Key>
__host__ __device__ inline size_t light_smem(uint32_t k) {
    const size_t NB = 1u << k;
    return light_cap<Key>() * (sizeof(Key) + 4 + 2) + NB * 4 + W_LOCAL * 64 * 4 + 64 * 4 +
           (2 * W_LOCAL + 2) * 4 + 64;
}

template <typename Key>
inline size_t heavy_smem(uint32_t k) {
    const size_t NB = 1u << k;
    return kHeavyChunk * (sizeof(Key) + 4 + 2) + 2 * NB * 4 + W_LOCAL * 64 * 4 + 64 * 4 +
           (2 * W_LOCAL + 2) * 4 + 64;
}

// Probe index entry of one bucket, x = its length.  32-bit keys: a bucket of
// at most three keys holds them all in y, z, w (its start is not needed to
// count matches); a longer one holds {len, start, first key, c0 | filter << 8}
// with c0 the entries equal to the first key and the filter of the other keys
// (filter_bit), so a query equal to the first key, any query against a bucket
// of one repeated key, and most queries matching no other key are answered
// without reading the edge array.  64-bit keys: {len, start, low and high
// half of the key} for a bucket of at most one key, {len, start, filter of
// all its keys (filter_bits64), low and high half} for a longer one, so that
// most queries matching none of its keys skip the edge array.  Unused key
// slots are 0.  A bucket longer than kRunBucket later gets its key-run
// summary in z, w.  `k` points at the bucket's first key.
template <typename Key>
__device__ __forceinline__ uint4 head_entry(uint32_t start, uint32_t end, const Key* k);

template <>
__device__ __forceinline__ uint4 head_entry<uint32_t>(uint32_t start, uint32_t end,
                                                      const uint32_t* k) {
    const uint32_t len = end - start;
    if (len <= 3)
        return make_uint4(len, len >= 1 ? k[0] : 0u, len >= 2 ? k[1] : 0u, len >= 3 ? k[2] : 0u);
    const uint32_t k0 = k[0];
    uint32_t c0 = 0, filt = 0;  // long buckets get their key runs in z, w instead
    if (len <= kRunBucket) {
        c0 = 1;
        // four keys per round, so that their loads overlap
#pragma unroll 1
        for (uint32_t i = 1; i < len; i += 4) {
            uint32_t kv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) kv[j] = i + j < len ? k[i + j] : k0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (i + j >= len) continue;
                if (kv[j] == k0) ++c0;
                else filt |= 1u << filter_bit(kv[j]);
            }
        }
    }
    return make_uint4(len, start, k0, c0 | filt << 8);
}

template <>
__device__ __forceinline__ uint4 head_entry<uint64_t>(uint32_t start, uint32_t end,
                                                      const uint64_t* k) {
    const uint32_t len = end - start;
    uint64_t z = len == 1 ? k[0] : 0ull;
    if (len >= 2 && len <= kRunBucket) {
#pragma unroll 1
        for (uint32_t i = 0; i < len; i += 4) {
            uint64_t kv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) kv[j] = i + j < len ? k[i + j] : k[0];
#pragma unroll
            for (int j = 0; j < 4; ++j) z |= filter_bits64(kv[j]);
        }
    }
    return make_uint4(len, start, (uint32_t)z, (uint32_t)(z >> 32));
}

// LDS of the per-bin key runs (after light_smem's layout, 16-byte aligned):
// the bin's long buckets (their range in the bin and bucket id), two counters
// and one 64-entry buffer per wave for the keys that differ from a bucket's
// first key.
template <typename Key>
struct LongLds {
    static constexpr uint32_t cap = light_cap<Key>() / (kRunBucket + 1) + 1;
    uint32_t* cnt;   // [0] long buckets of the bin, [1] of them left to the general pass
    uint32_t* lohi;  // [cap] lo | hi << 16: the bucket's range in the bin
    uint32_t* bkt;   // [cap] bucket id
    Key* wkey;       // [W_LOCAL * 64]
    uint16_t* wpos;  // [W_LOCAL * 64]
    __host__ __device__ static constexpr size_t bytes() {
        return 16 + 8 * cap + (sizeof(Key) + 2) * W_LOCAL * kWave + 32;
    }
    __device__ explicit LongLds(unsigned char* p) {
        cnt = (uint32_t*)p;
        lohi = cnt + 4;
        bkt = lohi + cap;
        wkey = (Key*)(((uintptr_t)(bkt + cap) + 15) & ~(uintptr_t)15);
        wpos = (uint16_t*)(wkey + W_LOCAL * kWave);
    }
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS bytes of a light bin that also builds its key runs.
template <typename Key>
__host__ __device__ inline size_t light_smem_index(uint32_t k) {
    return align16(light_smem<Key>(k)) + LongLds<Key>::bytes();
}

// Sort the 64 lanes' (key, position) pairs ascending (bitonic network over
// lane shuffles; positions are distinct, so the order is total).
template <typename Key>
__device__ __forceinline__ void wave_sort_pairs(Key& k, uint32_t& p) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (uint32_t size = 2; size <= (uint32_t)kWave; size <<= 1) {
#pragma unroll
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            const Key ok = __shfl_xor(k, (int)stride, kWave);
            const uint32_t op = __shfl_xor(p, (int)stride, kWave);
            const bool up = (lane & size) == 0;
            const bool lower = (lane & stride) == 0;
            const bool other_less = ok < k || (ok == k && op < p);
            if ((lower == up) ? other_less : !other_less) {
                k = ok;
                p = op;
            }
        }
    }
}

// Buckets whose index entry is built by one lane: up to 16 entries (rounds
// of four overlapped LDS reads).  Longer ones up to kRunBucket entries --
// common only when keys repeat many times -- are listed and built by groups
// of 32 lanes (bin_medium_heads) instead of one lane walking them in up to
// eight rounds.  (Groups of 16 lanes for buckets of 9-16 entries were faster
// only when keys repeat about 16 times, and slower below that.)
template <typename Key>
constexpr uint32_t head_lane_max() { return 16u; }

// A bucket's probe index entry, or its place in one of the bin's lists: the
// long buckets (more than kRunBucket entries; their entries are written with
// their key runs) and the medium ones (their entries are written by lane
// groups), med[] packing lo | len << 13 | v << 19 (v = local bucket).  k
// points at the bucket's first key in LDS.
template <typename Key>
__device__ __forceinline__ void note_bucket(const IndexOut& ix, const LongLds<Key>& lr,
                                            uint32_t* med, uint32_t v0, uint32_t v,
                                            uint32_t out, uint32_t lo, uint32_t hi,
                                            const Key* k) {
    const uint32_t len = hi - lo;
    if (len > kRunBucket) {
        const uint32_t t = atomicAdd(&lr.cnt[0], 1u);
        lr.lohi[t] = lo | (hi << 16);
        lr.bkt[t] = v0 + v;
    } else if (len > head_lane_max<Key>()) {
        med[atomicAdd(&lr.cnt[2], 1u)] = lo | (len << 13) | (v << 19);
    } else {
        ix.head[v0 + v] = head_entry<Key>(out + lo, out + hi, k);
    }
}

// OR over each row of 16 lanes, left in the row's last lane (lanes 15, 31,
// 47, 63): four DPP row shifts (a lane shifted in from outside the row reads
// 0).  Whole wave.
__device__ __forceinline__ uint32_t row_or16(uint32_t f) {
    f |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)f, 0x111, 0xf, 0xf, false);  // row_shr:1
    f |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)f, 0x112, 0xf, 0xf, false);  // row_shr:2
    f |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)f, 0x114, 0xf, 0xf, false);  // row_shr:4
    f |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)f, 0x118, 0xf, 0xf, false);  // row_shr:8
    return f;
}

// The OR of group g's lanes (groups of G = 16 or 32 lanes), from the rows'
// ORs; uniform values, selected per lane.
template <uint32_t G>
__device__ __forceinline__ uint32_t group_or(uint32_t f, uint32_t g) {
    const uint32_t r = row_or16(f);
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)r, 15);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)r, 31);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)r, 47);
    const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)r, 63);
    if constexpr (G == 16) return g == 0 ? a : g == 1 ? b : g == 2 ? c : d;
    else return g == 0 ? (a | b) : (c | d);
}

// Index entries of the medium buckets in list[0, n), whose lengths are at
// most G: each wave takes 64 / G buckets at a time, lane s of group g holding
// key s of its bucket; the first key's count is a ballot and the filter an
// OR over the group -- the same entry head_entry builds with one lane.
template <typename Key, uint32_t G>
__device__ __forceinline__ void medium_heads_by(const IndexOut& ix, const uint32_t* list,
                                                uint32_t n, const Key* skeys, uint32_t out,
                                                uint32_t v0) {
    constexpr uint32_t PER = kWave / G;
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t g = lane / G, s = lane % G;
    for (uint32_t j0 = w * PER; j0 < n; j0 += W_LOCAL * PER) {  // uniform per wave
        const uint32_t j = j0 + g;
        const bool have = j < n;
        const uint32_t e = have ? list[j] : 0u;
        const uint32_t lo = e & 0x1fffu, len = (e >> 13) & 0x3fu, v = e >> 19;
        const bool in = have && s < len;
        const Key k0 = skeys[lo];
        const Key kx = in ? skeys[lo + s] : k0;
        if constexpr (sizeof(Key) == 4) {
            const uint64_t eq = ballot(in && kx == k0);
            const uint32_t c0 = (uint32_t)__popcll((eq >> (g * G)) & ((1ull << G) - 1ull));
            const uint32_t f =
                group_or<G>((in && kx != k0) ? (1u << filter_bit((uint32_t)kx)) : 0u, g);
            if (have && s == 0) ix.head[v0 + v] = make_uint4(len, out + lo, (uint32_t)k0, c0 | f << 8);
        } else {
            const uint64_t z = in ? filter_bits64((uint64_t)kx) : 0ull;
            const uint32_t zl = group_or<G>((uint32_t)z, g), zh = group_or<G>((uint32_t)(z >> 32), g);
            if (have && s == 0) ix.head[v0 + v] = make_uint4(len, out + lo, zl, zh);
        }
    }
}

// Index entries of the bin's medium buckets (more than head_lane_max and at
// most kRunBucket entries).  Called by whole waves after a barrier that
// follows the list's construction.
template <typename Key>
__device__ __forceinline__ void bin_medium_heads(const IndexOut& ix, const LongLds<Key>& lr,
                                                 const uint32_t* med, const Key* skeys,
                                                 uint32_t out, uint32_t v0) {
    static_assert(kRunBucket <= 32u, "a medium bucket fits a group of 32 lanes");
    medium_heads_by<Key, 32>(ix, med, lr.cnt[2], skeys, out, v0);
}

// Key runs and index entry of one long bucket, by one wave: its entries are
// keys[lo, hi) with ids ids_[lo, hi) (in LDS or in global memory), its first
// edge is at st, its bucket id b.  The entries equal to the bucket's first
// key (the lead key) form one run; the others, when there are at most 64, are
// sorted across the wave's lanes and cut into runs, and the lead run is
// slotted in among them.  bk / bp: the wave's 64-entry LDS buffers.  Returns
// false, having written nothing, when more than 64 entries differ from the
// lead key (uniform across the wave).
template <typename Key>
__device__ __forceinline__ bool wave_bucket_runs(const IndexOut& ix, const Key* keys,
                                                 const uint32_t* ids_, uint32_t lo, uint32_t hi,
                                                 uint32_t st, uint32_t b, Key* bk, uint16_t* bp) {
    const uint32_t lane = lane_id();
    Key* rkey = (Key*)ix.runs.run_key;
    uint32_t* rend = ix.runs.run_end;
    uint32_t* kperm = ix.runs.kperm;
    const uint32_t len = hi - lo;
    const Key lead = keys[lo];
    uint32_t no = 0;  // entries whose key differs from the lead key
    for (uint32_t c = lo; c < hi; c += kWave) {
        const uint32_t p = c + lane;
        const Key x = p < hi ? keys[p] : lead;
        const bool o = x != lead;
        const uint64_t bal = ballot(o);
        const uint32_t slot = no + mbcnt(bal);
        if (o && slot < (uint32_t)kWave) {
            bk[slot] = x;
            bp[slot] = (uint16_t)(p - lo);
        }
        no += (uint32_t)__popcll(bal);
        if (no > (uint32_t)kWave) return false;  // too many others: stop reading
    }
    if (no == 0) {  // one key: its ids are the edge array's own
        if (lane == 0) {
            rkey[st] = lead;
            rend[st] = len;
            ix.head[b] = make_uint4(len, st, 1u, sizeof(Key) == 4 ? (uint32_t)lead : 0u);
        }
        return true;
    }
    // the buffer written above is read by other lanes of the same wave:
    // LDS executes a wave's operations in order; keep the compiler's too
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool valid = lane < no;
    Key k = valid ? bk[lane] : (Key)~(Key)0;
    uint32_t p = valid ? (uint32_t)bp[lane] : 0xffffffffu;
    wave_sort_pairs<Key>(k, p);
    const Key kprev = __shfl_up(k, 1, kWave);
    const Key knext = __shfl_down(k, 1, kWave);
    const bool first = valid && (lane == 0 || kprev != k);
    const bool last = valid && (lane + 1 == no || knext != k);
    const bool below = valid && k < lead;
    const uint64_t fb = ballot(first), lb = ballot(below);
    const uint32_t nless = (uint32_t)__popcll(lb);       // others below the lead key
    const uint32_t rl = (uint32_t)__popcll(fb & lb);     // runs below the lead key
    const uint32_t clead = len - no;
    const uint32_t r = mbcnt(fb) + (first ? 1u : 0u) - 1u + (below ? 0u : 1u);
    if (valid) kperm[st + lane + (below ? 0u : clead)] = ids_[lo + p];
    if (first) rkey[st + r] = k;
    if (last) rend[st + r] = lane + 1 + (below ? 0u : clead);
    if (lane == 0) {
        rkey[st + rl] = lead;
        rend[st + rl] = nless + clead;
        ix.head[b] = make_uint4(len, st, (uint32_t)__popcll(fb) + 1u, 0u);
    }
    // the lead key's ids, in bucket order, after the smaller keys' runs
    uint32_t done = 0;
    for (uint32_t c = lo; c < hi; c += kWave) {
        const uint32_t q = c + lane;
        const bool isl = q < hi && keys[q] == lead;
        const uint64_t bal = ballot(isl);
        if (isl) kperm[st + nless + done + mbcnt(bal)] = ids_[q];
        done += (uint32_t)__popcll(bal);
    }
    return true;
}

// Key runs of the long buckets of a bin held in LDS (skeys / sids in bucket
// order, the bin's first edge at `out`), one wave per bucket.  The entries
// equal to the bucket's first key (the lead key) form one run; the others,
// when there are at most 64, are sorted across the wave's lanes and cut into
// runs, and the lead run is slotted in among them.  A bucket with more other
// keys is listed for the general pass.  Whole workgroup; barriers.
template <typename Key>
__device__ __forceinline__ void bin_long_runs(const IndexOut& ix, const LongLds<Key>& lr,
                                              const uint32_t* med, const Key* skeys,
                                              const uint32_t* sids, uint32_t out, uint32_t g,
                                              uint32_t v0) {
    __syncthreads();
    bin_medium_heads<Key>(ix, lr, med, skeys, out, v0);
    const uint32_t nl = lr.cnt[0];
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    Key* bk = lr.wkey + w * kWave;
    uint16_t* bp = lr.wpos + w * kWave;
    for (uint32_t j = w; j < nl; j += W_LOCAL) {
        const uint32_t lh = lr.lohi[j], lo = lh & 0xffffu, hi = lh >> 16;
        const uint32_t b = lr.bkt[j];
        if (!wave_bucket_runs<Key>(ix, skeys, sids, lo, hi, out + lo, b, bk, bp) && lane == 0)
            ix.gen_list[gen_region(out, g) + atomicAdd(&lr.cnt[1], 1u)] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) ix.gen_cnt[g] = lr.cnt[1];
}

// Build one bin of L <= light_cap<Key>() keys whose buckets are [v0, v0 + nb) with
// nb <= 2^k.  Entry e (e < L) of the bin is src_keys[e], with id src_ids[e]
// (or id_base + e when src_ids is null).  The bin's keys and ids go to
// ekeys/ids[out + p] for p < L, sorted by bucket with ids ascending inside a
// bucket, and offsets[v0 + v] = out + (start of bucket v in the bin).
// Usual case (every bucket of the bin holds at most kFixMax keys, or any order
// is allowed): LDS
// counting sort with atomic cursors, then an insertion sort by id inside each
// bucket (skipped with any_order: order inside a bucket is then unspecified).
// Otherwise the bin (in id order) is stably ranked by local bucket.
// When ix.head is not null it also receives each bucket's probe index entry.
// `bucket_of(key, e)` gives the local bucket (< nb) of entry e.
// Called by a whole workgroup of kLocalThreads threads.
template <typename Key, typename BucketOf>
__device__ __forceinline__ void light_bin_body_by(const Key* __restrict__ src_keys,
                                                  const uint32_t* __restrict__ src_ids,
                                                  uint32_t id_base, uint32_t L, uint32_t out,
                                                  uint32_t v0, uint32_t k, uint32_t nb,
                                                  BucketOf bucket_of,
                                                  uint32_t* __restrict__ offsets,
                                                  const IndexOut& ix, uint32_t* __restrict__ ids,
                                                  Key* __restrict__ ekeys, unsigned char* smem,
                                                  bool any_order) {
    constexpr int IT = light_items<Key>();
    constexpr uint32_t kLightCap = light_cap<Key>();
    const uint32_t NB = 1u << k;
    Key* skeys = (Key*)smem;
    uint32_t* sids = (uint32_t*)(skeys + kLightCap);
    uint16_t* sb = (uint16_t*)(sids + kLightCap);
    // the bucket sort's scratch holds the list of medium buckets afterwards
    // (at most kLightCap / (head_lane_max + 1) of them; room for kLightCap / 2)
    static_assert(kLightCap <= 8192u, "a medium-list entry holds lo in 13 bits");
    uint32_t* med = (uint32_t*)sb;
    uint32_t* cnt = (uint32_t*)(sb + kLightCap);  // NB
    uint32_t* wcnt = cnt + NB;                     // W * 64
    uint32_t* dstart = wcnt + W_LOCAL * 64;        // 64
    uint32_t* tmp = dstart + 64;
    // the bin's long buckets, when the probe index is written
    const LongLds<Key> lr(smem + align16(light_smem<Key>(k)));
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    // balance the bin over the waves in whole rounds of 64
    const uint32_t wchunk = (((L + W_LOCAL - 1) / W_LOCAL) + kWave - 1) & ~(uint32_t)(kWave - 1);
    const uint32_t wb = w * wchunk;
    const uint32_t mylen = L > wb ? ((L - wb < wchunk) ? L - wb : wchunk) : 0u;
    const uint32_t rounds = (mylen + kWave - 1) / kWave;

    Key kk[IT];
    uint32_t id[IT], b[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t e = wb + r * kWave + lane;
        if ((uint32_t)r < rounds && r * kWave + lane < mylen) {
            kk[r] = src_keys[e];
            id[r] = src_ids ? src_ids[e] : id_base + e;
        } else {
            kk[r] = 0;
            id[r] = 0;
        }
    }
    for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads) cnt[i] = 0;
    if (ix.head && threadIdx.x < 3) lr.cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) dstart[0] = 0;  // list of multi-entry buckets (stable path)
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        if ((uint32_t)r < rounds && r * kWave + lane < mylen) {
            b[r] = bucket_of(kk[r], wb + r * kWave + lane);
            atomicAdd(&cnt[b[r]], 1u);
        } else {
            b[r] = NB;
        }
    }
    __syncthreads();
    // bucket starts (in place) and the largest bucket of the bin
    const uint32_t maxc = scan_counts_max(cnt, NB, tmp);
    if (maxc <= kFixMax || any_order) {
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            if (b[r] < NB) {
                const uint32_t slot = atomicAdd(&cnt[b[r]], 1u);
                skeys[slot] = kk[r];
                sids[slot] = id[r];
            }
        }
        __syncthreads();
        // cnt[v] is now the end of bucket v; ids are put back in ascending
        // order inside each (short) bucket unless any order is allowed.  The
        // buckets of two or more entries are listed first (in the bucket
        // sort's scratch, unused on this path: at most L / 2 of them, packed
        // lo | len << 16), so that every lane of the sorting pass has one.
        if (!any_order) {
            uint32_t* multi = (uint32_t*)sb;
            for (uint32_t v = threadIdx.x; v < NB; v += kLocalThreads) {
                const uint32_t lo = v ? cnt[v - 1] : 0u, hi = cnt[v];
                if (hi - lo >= 2) multi[atomicAdd(&dstart[0], 1u)] = lo | ((hi - lo) << 16);
            }
            __syncthreads();
            const uint32_t nmulti = dstart[0];
            for (uint32_t j = threadIdx.x; j < nmulti; j += kLocalThreads) {
                const uint32_t lo = multi[j] & 0xffffu, len = multi[j] >> 16, hi = lo + len;
                if (len <= 8) {
                    sort8_by_id<Key>(sids + lo, skeys + lo, len);
                    continue;
                }
                for (uint32_t i = lo + 1; i < hi; ++i) {
                    const uint32_t idv = sids[i];
                    const Key kv = skeys[i];
                    uint32_t j2 = i;
                    while (j2 > lo && sids[j2 - 1] > idv) {
                        sids[j2] = sids[j2 - 1];
                        skeys[j2] = skeys[j2 - 1];
                        --j2;
                    }
                    sids[j2] = idv;
                    skeys[j2] = kv;
                }
            }
        }
        __syncthreads();
        for (uint32_t v = threadIdx.x; v < nb; v += kLocalThreads) {
            const uint32_t lo = v ? cnt[v - 1] : 0u, hi = cnt[v];
            offsets[v0 + v] = out + lo;
            if (ix.head) note_bucket<Key>(ix, lr, med, v0, v, out, lo, hi, skeys + lo);
        }
    } else {
        sort_chunk_by_bucket<Key, IT>(kk, id, b, rounds, L, wchunk, k, skeys, sids, sb, wcnt,
                                      dstart, tmp);
        __syncthreads();
        for (uint32_t v = threadIdx.x; v < nb; v += kLocalThreads) {
            const uint32_t lo = cnt[v], hi = (v + 1 < NB) ? cnt[v + 1] : L;
            offsets[v0 + v] = out + lo;
            if (ix.head) note_bucket<Key>(ix, lr, med, v0, v, out, lo, hi, skeys + lo);
        }
    }
    for (uint32_t p = threadIdx.x; p < L; p += kLocalThreads) {
        ekeys[out + p] = skeys[p];
        ids[out + p] = sids[p];
    }
    if (ix.head) bin_long_runs<Key>(ix, lr, med, skeys, sids, out, v0 >> k, v0);
}

// The usual bin: buckets [v0, v0 + nb) of the table's hash function.
template <typename Key>
__device__ __forceinline__ void light_bin_body(const Key* __restrict__ src_keys,
                                               const uint32_t* __restrict__ src_ids,
                                               uint32_t id_base, uint32_t L, uint32_t out,
                                               uint32_t v0, uint32_t k, uint32_t nb,
                                               const typename KeyTraits<Key>::Params& hp,
                                               uint32_t* __restrict__ offsets,
                                               const IndexOut& ix,
                                               uint32_t* __restrict__ ids, Key* __restrict__ ekeys,
                                               unsigned char* smem, bool any_order = false) {
    light_bin_body_by<Key>(
        src_keys, src_ids, id_base, L, out, v0, k, nb,
        [&](Key key, uint32_t) { return KeyTraits<Key>::bucket(key, hp) - v0; }, offsets, ix, ids,
        ekeys, smem, any_order);
}

// Pointers into the heavy_smem layout.
template <typename Key>
struct HeavyLds {
    Key* skeys;
    uint32_t* sids;
    uint16_t* sb;
    uint32_t *cur, *tcnt, *wcnt, *dstart, *tmp;
    __device__ HeavyLds(unsigned char* smem, uint32_t NB) {
        skeys = (Key*)smem;
        sids = (uint32_t*)(skeys + kHeavyChunk);
        sb = (uint16_t*)(sids + kHeavyChunk);
        cur = (uint32_t*)(sb + kHeavyChunk);  // NB: running cursors
        tcnt = cur + NB;                      // NB: chunk-local bucket starts
        wcnt = tcnt + NB;
        dstart = wcnt + W_LOCAL * 64;
        tmp = dstart + 64;
    }
};

// Place L entries (arriving in id order) of one bin, chunk by chunk, in
// order: each chunk is sorted by bucket in LDS and written at the running
// per-bucket cursors cur[0 .. 2^k), which hold absolute edge positions on
// entry and are advanced past the placed entries on return.  Writes outside
// [lo, hi) are dropped (they cannot happen for consistent counts).  With
// any_order a chunk is grouped by bucket with one returning LDS atomic per
// key (the lanes sharing the wave's first lane's bucket take one for the
// group) instead of two stable ranking passes.  Uses the heavy_smem layout;
// whole workgroup.
template <typename Key>
__device__ __forceinline__ void place_in_chunks(const Key* __restrict__ src_keys,
                                                const uint32_t* __restrict__ src_ids,
                                                uint32_t id_base, uint32_t L, uint32_t lo,
                                                uint32_t hi, uint32_t v0, uint32_t k,
                                                const typename KeyTraits<Key>::Params& hp,
                                                uint32_t* __restrict__ ids,
                                                Key* __restrict__ ekeys, unsigned char* smem,
                                                bool any_order = false) {
    constexpr int IT = kHeavyItems;
    constexpr uint32_t CAP = kHeavyChunk;
    const uint32_t NB = 1u << k;
    const HeavyLds<Key> m(smem, NB);
    Key* skeys = m.skeys;
    uint32_t* sids = m.sids;
    uint16_t* sb = m.sb;
    uint32_t *cur = m.cur, *tcnt = m.tcnt, *wcnt = m.wcnt, *dstart = m.dstart, *tmp = m.tmp;
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t nchunk = (uint32_t)(((uint64_t)L + CAP - 1) / CAP);
    for (uint32_t ci = 0; ci < nchunk; ++ci) {
        const uint32_t c0 = ci * CAP;
        const uint32_t cl = (L - c0 < CAP) ? L - c0 : CAP;
        const uint32_t wchunk =
            (((cl + W_LOCAL - 1) / W_LOCAL) + kWave - 1) & ~(uint32_t)(kWave - 1);
        const uint32_t wb = w * wchunk;
        const uint32_t mylen = cl > wb ? ((cl - wb < wchunk) ? cl - wb : wchunk) : 0u;
        const uint32_t rounds = (mylen + kWave - 1) / kWave;
        Key kk[IT];
        uint32_t id[IT], b[IT];
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const uint32_t e = c0 + wb + r * kWave + lane;
            if ((uint32_t)r < rounds && r * kWave + lane < mylen) {
                kk[r] = src_keys[e];
                id[r] = src_ids ? src_ids[e] : id_base + e;
            } else {
                kk[r] = 0;
                id[r] = 0;
            }
        }
        for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads) tcnt[i] = 0;
        __syncthreads();
        // bins this large usually hold a hot key: the lanes whose bucket
        // equals the wave's first lane's add their count with one atomic (a
        // single LDS address hit by every lane would serialise 64 ways), the
        // others add one each
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const bool valid = (uint32_t)r < rounds && r * kWave + lane < mylen;
            b[r] = valid ? KeyTraits<Key>::bucket(kk[r], hp) - v0 : NB;
            const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b[r]);
            const bool first = valid && b[r] == b0;
            const uint64_t same = ballot(first);
            if (first) {
                if (mbcnt(same) == 0) atomicAdd(&tcnt[b0], (uint32_t)__popcll(same));
            } else if (valid) {
                atomicAdd(&tcnt[b[r]], 1u);
            }
        }
        if (any_order) {
            __syncthreads();
            // chunk-local bucket starts; the slots taken below turn them into
            // bucket ends, and a bucket starts where the one before it ends
            scan_counts(tcnt, NB, 0u, tmp);
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                const bool valid = b[r] < NB;
                const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b[r]);
                const bool first = valid && b[r] == b0;
                const uint64_t same = ballot(first);
                uint32_t slot = 0;
                if (first) {
                    uint32_t base = 0;
                    if (mbcnt(same) == 0) base = atomicAdd(&tcnt[b0], (uint32_t)__popcll(same));
                    slot = (uint32_t)__shfl((int)base, (int)__builtin_ctzll(same), kWave) +
                           mbcnt(same);
                } else if (valid) {
                    slot = atomicAdd(&tcnt[b[r]], 1u);
                }
                if (valid) {
                    skeys[slot] = kk[r];
                    sids[slot] = id[r];
                    sb[slot] = (uint16_t)b[r];
                }
            }
            __syncthreads();
            for (uint32_t p = threadIdx.x; p < cl; p += kLocalThreads) {
                const uint32_t bb = sb[p];
                const uint32_t st = bb ? tcnt[bb - 1] : 0u;
                const uint32_t o = cur[bb] + (p - st);
                if (o - lo < hi - lo) {
                    ekeys[o] = skeys[p];
                    ids[o] = sids[p];
                }
            }
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads)
                cur[i] += tcnt[i] - (i ? tcnt[i - 1] : 0u);
            __syncthreads();
            continue;
        }
        sort_chunk_by_bucket<Key, IT>(kk, id, b, rounds, cl, wchunk, k, skeys, sids, sb, wcnt,
                                      dstart, tmp);
        __syncthreads();
        // chunk-local bucket starts (exclusive scan of tcnt)
        scan_counts(tcnt, NB, 0u, tmp);
        for (uint32_t p = threadIdx.x; p < cl; p += kLocalThreads) {
            const uint32_t bb = sb[p];
            const uint32_t o = cur[bb] + (p - tcnt[bb]);
            if (o - lo < hi - lo) {
                ekeys[o] = skeys[p];
                ids[o] = sids[p];
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads) {
            const uint32_t nxt = (i + 1 < NB) ? tcnt[i + 1] : cl;
            cur[i] += nxt - tcnt[i];
        }
        __syncthreads();
    }
}

// The same for a bin of any size (arriving in id order) in one workgroup:
// keys counted per bucket first, then placed with place_in_chunks, so
// placement stays stable.
template <typename Key>
__device__ __forceinline__ void heavy_bin_body(const Key* __restrict__ src_keys,
                                               const uint32_t* __restrict__ src_ids,
                                               uint32_t id_base, uint32_t L, uint32_t out,
                                               uint32_t v0, uint32_t k, uint32_t nb,
                                               const typename KeyTraits<Key>::Params& hp,
                                               uint32_t* __restrict__ offsets,
                                               const IndexOut& ix,
                                               uint32_t* __restrict__ ids, Key* __restrict__ ekeys,
                                               unsigned char* smem, bool any_order = false) {
    const uint32_t NB = 1u << k;
    const HeavyLds<Key> m(smem, NB);
    uint32_t *cur = m.cur, *tmp = m.tmp;

    for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads) cur[i] = 0;
    __syncthreads();
    // lanes sharing the first active lane's bucket (a hot key) count with one
    // LDS atomic, the others one each
    for (uint32_t i = threadIdx.x; i < L; i += kLocalThreads) {
        const uint32_t b = KeyTraits<Key>::bucket(src_keys[i], hp) - v0;
        const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b);
        const uint64_t same = ballot(b == b0);
        if (b != b0) atomicAdd(&cur[b], 1u);
        else if (mbcnt(same) == 0) atomicAdd(&cur[b0], (uint32_t)__popcll(same));
    }
    __syncthreads();
    scan_counts(cur, NB, out, tmp);
    for (uint32_t i = threadIdx.x; i < nb; i += kLocalThreads) offsets[v0 + i] = cur[i];
    place_in_chunks<Key>(src_keys, src_ids, id_base, L, out, out + L, v0, k, hp, ids, ekeys,
                         smem, any_order);
    // cur[v] is now the end of bucket v; the bin's edges are in ekeys.  Long
    // buckets are listed for the general pass, which builds their key runs.
    if (ix.head) {
        uint32_t* nlisted = tmp + 2 * W_LOCAL + 2;  // inside heavy_smem's padding
        if (threadIdx.x == 0) *nlisted = 0;
        __syncthreads();
        for (uint32_t v = threadIdx.x; v < nb; v += kLocalThreads) {
            const uint32_t lo = v ? cur[v - 1] : out;
            if (cur[v] - lo > kRunBucket)
                ix.gen_list[gen_region(out, v0 >> k) + atomicAdd(nlisted, 1u)] = v0 + v;
            else
                ix.head[v0 + v] = head_entry<Key>(lo, cur[v], ekeys + lo);
        }
        __syncthreads();
        if (threadIdx.x == 0) ix.gen_cnt[v0 >> k] = *nlisted;
    }
}

}  // namespace v2dev
}  // namespace hg
