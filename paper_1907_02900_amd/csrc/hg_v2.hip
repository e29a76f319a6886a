// HashGraph-V2 (Alg. 2) on gfx950.
//
// The paper's idea -- first move keys into bins of contiguous bucket ranges so
// that the final placement is cache-local -- mapped onto CDNA4 without any
// global atomics:
//   * a final bin is a power-of-two range of 2^k buckets holding about 4096
//     32-bit keys (2048 64-bit keys) on average, so that its keys, ids and
//     bucket counters fit in the LDS of one 512-thread workgroup;
//   * keys reach their final bin by one or two stable partition passes over a
//     digit (a bit-field) of the bucket index.  Each pass is: per-tile digit
//     histograms (LDS), a segmented column scan of the tile x digit matrix
//     (giving every tile an exact base per digit: deterministic, no atomics),
//     and a partition kernel that ranks a tile's keys by digit with wave64
//     ballots and writes digit-contiguous runs;
//   * one workgroup per final bin counts, scans and stably places the bin's
//     keys in LDS (two LSD ranking passes over the local bucket index) and
//     writes the bin's edge segment and offsets with coalesced stores.  Bins
//     larger than LDS (heavy skew only) are listed on the device and handled
//     by a second kernel in chunks with running per-bucket cursors.
// Every pass keeps input order among equal digits, so ids come out ascending
// inside each bucket: the result is the stable layout, entry for entry.
//
// Stable ranking (rank_stable) finds equal digits in a round of 64 items with
// one ballot per digit bit and keeps per-wave running counts in LDS, updated
// with non-returning atomics so that rounds do not wait on each other.
#include "hg_v2_device.h"

namespace hg {

namespace {

using namespace v2dev;

// Segments of the source array, each cut into tiles of kPartTile entries, and
// the tiles grouped into chunks of `ch` consecutive tiles for the column scan.
struct Segs {
    uint32_t* seg_start;     // [S+1]
    uint32_t* tile_prefix;   // [S+1]
    uint32_t* chunk_prefix;  // [S+1]
    uint32_t S;
    uint32_t ch;
};

// largest s in [0, S) with pre[s] <= x (pre non-decreasing, pre[0] = 0)
__device__ __forceinline__ uint32_t find_seg(const uint32_t* __restrict__ pre, uint32_t S,
                                             uint32_t x) {
    uint32_t lo = 0, hi = S;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool locate_tile(const Segs& g, uint32_t t, uint32_t& seg,
                                            uint32_t& begin, uint32_t& end) {
    if (t >= g.tile_prefix[g.S]) return false;
    seg = find_seg(g.tile_prefix, g.S, t);
    begin = g.seg_start[seg] + (t - g.tile_prefix[seg]) * kPartTile;
    const uint32_t se = g.seg_start[seg + 1];
    end = (se - begin > kPartTile) ? begin + kPartTile : se;
    return true;
}

// (xcd_tile: the runs that neighbouring tiles write for a digit meet in
// one XCD's L2)

// ---------------------------------------------------- tile histograms -----

// ID_DIGIT: the digit is a bit-field of the entry's id (ids[i] >> shift)
// instead of the bucket of its key (the scatter by a permutation below).
// QUERIES: the same code, instantiated apart for grouping a probe's queries
// so that kernel traces tell it from the build's passes (also below).
template <typename Key, bool ID_DIGIT = false, bool QUERIES = false>
__global__ __launch_bounds__(kPartThreads) void k_tile_hist(const Key* __restrict__ keys, Segs g,
                                                            typename KeyTraits<Key>::Params hp,
                                                            uint32_t shift, uint32_t bits,
                                                            uint32_t* __restrict__ mat,
                                                            uint32_t tiles_ub,
                                                            const uint32_t* __restrict__ ids = nullptr) {
    extern __shared__ uint32_t cnt[];
    const uint32_t D = 1u << bits;
    const uint32_t t = xcd_tile(blockIdx.x, tiles_ub);
    uint32_t seg, begin, end;
    if (!locate_tile(g, t, seg, begin, end)) return;
    for (uint32_t d = threadIdx.x; d < D; d += kPartThreads) cnt[d] = 0;
    constexpr int IT = kPartItems;
    Key k[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t i = begin + r * kPartThreads + threadIdx.x;
        if (ID_DIGIT) k[r] = (i < end) ? (Key)ids[i] : (Key)0;
        else k[r] = (i < end) ? keys[i] : (Key)0;
    }
    __syncthreads();
    const uint32_t mask = D - 1;
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t i = begin + r * kPartThreads + threadIdx.x;
        const uint32_t v = ID_DIGIT ? (uint32_t)k[r] : KeyTraits<Key>::bucket(k[r], hp);
        if (i < end) atomicAdd(&cnt[(v >> shift) & mask], 1u);
    }
    __syncthreads();
    uint32_t* row = mat + (size_t)t * D;
    for (uint32_t d = threadIdx.x; d < D; d += kPartThreads) row[d] = cnt[d];
}

// ------------------------------------- segmented column scan of [tile][digit]
// base(t, d) = seg_start[s] + sum_{d' < d} total_s(d') + sum_{t' < t in s} M[t'][d]
// i.e. the exclusive prefix in (segment, digit, tile) order: where tile t's
// keys of digit d go in the stably partitioned output.

__device__ __forceinline__ bool locate_chunk(const Segs& g, uint32_t c, uint32_t& seg,
                                             uint32_t& t0, uint32_t& t1) {
    if (c >= g.chunk_prefix[g.S]) return false;
    seg = find_seg(g.chunk_prefix, g.S, c);
    t0 = g.tile_prefix[seg] + (c - g.chunk_prefix[seg]) * g.ch;
    const uint32_t te = g.tile_prefix[seg + 1];
    t1 = (te - t0 > g.ch) ? t0 + g.ch : te;
    return true;
}

__global__ __launch_bounds__(256) void k_colscan_reduce(const uint32_t* __restrict__ mat, Segs g,
                                                        uint32_t D, uint32_t* __restrict__ csum) {
    uint32_t seg, t0, t1;
    if (!locate_chunk(g, blockIdx.x, seg, t0, t1)) return;
    for (uint32_t d = threadIdx.x; d < D; d += 256) {
        uint32_t s = 0;
        uint32_t t = t0;
        for (; t + 8 <= t1; t += 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = mat[(size_t)(t + u) * D + d];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; t < t1; ++t) s += mat[(size_t)t * D + d];
        csum[(size_t)blockIdx.x * D + d] = s;
    }
}

// One workgroup per segment: digit totals, their exclusive scan, then each
// digit walks its chunks turning chunk sums into chunk bases.
__global__ __launch_bounds__(256) void k_colscan_seg(Segs g, uint32_t D,
                                                     uint32_t* __restrict__ csum) {
    __shared__ uint32_t tmp[256 / kWave + 1];
    const uint32_t s = blockIdx.x;
    const uint32_t c0 = g.chunk_prefix[s], c1 = g.chunk_prefix[s + 1];
    if (c0 == c1) return;
    const uint32_t per = (D + 255) / 256;  // <= 8 (D <= 2048)
    const uint32_t d0 = threadIdx.x * per;
    uint32_t tot[8];
    uint32_t mine = 0;
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t d = d0 + j;
        uint32_t acc = 0;
        if (d < D)
            for (uint32_t c = c0; c < c1; ++c) acc += csum[(size_t)c * D + d];
        tot[j] = acc;
        mine += acc;
    }
    uint32_t all;
    uint32_t run = g.seg_start[s] + block_excl_scan<256>(mine, tmp, &all);
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t d = d0 + j;
        if (d < D) {
            uint32_t r = run;
            for (uint32_t c = c0; c < c1; ++c) {
                const uint32_t v = csum[(size_t)c * D + d];
                csum[(size_t)c * D + d] = r;
                r += v;
            }
        }
        run += tot[j];
    }
}

__global__ __launch_bounds__(256) void k_colscan_down(uint32_t* __restrict__ mat, Segs g, uint32_t D,
                                                      const uint32_t* __restrict__ csum) {
    uint32_t seg, t0, t1;
    if (!locate_chunk(g, blockIdx.x, seg, t0, t1)) return;
    for (uint32_t d = threadIdx.x; d < D; d += 256) {
        uint32_t r = csum[(size_t)blockIdx.x * D + d];
        uint32_t t = t0;
        for (; t + 8 <= t1; t += 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = mat[(size_t)(t + u) * D + d];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                mat[(size_t)(t + u) * D + d] = r;
                r += v[u];
            }
        }
        for (; t < t1; ++t) {
            const uint32_t v = mat[(size_t)t * D + d];
            mat[(size_t)t * D + d] = r;
            r += v;
        }
    }
}

// ------------------------------------------------------------ partition ---

// Stable partition of one tile by a digit of the bucket index.  Writes every
// entry to base(tile, digit) + its rank among the tile's entries of that
// digit.
// STABLE: entries of equal digit keep their order (rank_stable); otherwise
// their order inside a run is unspecified (rank_any, no ballots).
template <typename Key, bool HAS_IDS, bool STABLE, bool ID_DIGIT = false, bool QUERIES = false>
__global__ __launch_bounds__(kPartThreads) void k_tile_partition(
    const Key* __restrict__ src_keys, const uint32_t* __restrict__ src_ids,
    Key* __restrict__ dst_keys, uint32_t* __restrict__ dst_ids, Segs g,
    typename KeyTraits<Key>::Params hp, uint32_t shift, uint32_t bits,
    const uint32_t* __restrict__ base, uint32_t tiles_ub) {
    constexpr int IT = kPartItems;
    const uint32_t D = 1u << bits;
    extern __shared__ __align__(16) unsigned char smem[];
    Key* skeys = (Key*)smem;
    uint32_t* sids = (uint32_t*)(skeys + kPartTile);
    uint16_t* sdig = (uint16_t*)(sids + kPartTile);
    uint32_t* wcnt = (uint32_t*)(sdig + kPartTile);
    uint32_t* dstart = wcnt + W_PART * D;
    uint32_t* tbase = dstart + D;
    uint32_t* tmp = tbase + D;

    const uint32_t t = xcd_tile(blockIdx.x, tiles_ub);
    uint32_t seg, begin, end;
    if (!locate_tile(g, t, seg, begin, end)) return;
    const uint32_t cnt = end - begin;
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t mask = D - 1;
    const uint32_t wbase = w * (kWave * IT);

    Key k[IT];
    uint32_t id[IT], dig[IT], pos[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t e = wbase + r * kWave + lane;
        if (e < cnt) {
            k[r] = src_keys[begin + e];
            id[r] = HAS_IDS ? src_ids[begin + e] : begin + e;
        } else {
            k[r] = 0;
            id[r] = 0;
        }
    }
    // the tile's digit bases, loaded now so that their latency overlaps the
    // ranking (D <= 2048: at most kRowPer per thread)
    constexpr int kRowPer = (1 << kMaxDigitBits) / kPartThreads;
    const uint32_t* row = base + (size_t)t * D;
    uint32_t rowv[kRowPer];
#pragma unroll
    for (int j = 0; j < kRowPer; ++j) {
        const uint32_t d = threadIdx.x + j * kPartThreads;
        rowv[j] = d < D ? row[d] : 0u;
    }
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t e = wbase + r * kWave + lane;
        const uint32_t v = ID_DIGIT ? id[r] : KeyTraits<Key>::bucket(k[r], hp);
        dig[r] = (e < cnt) ? ((v >> shift) & mask) : D;
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
            skeys[pos[r]] = k[r];
            sids[pos[r]] = id[r];
            sdig[pos[r]] = (uint16_t)dig[r];
        }
    }
    __syncthreads();
    // every output lies inside this segment's range; the guard keeps a
    // corrupted base from turning into a stray store
    const uint32_t seg_lo = g.seg_start[seg], seg_len = g.seg_start[seg + 1] - seg_lo;
    for (uint32_t p = threadIdx.x; p < cnt; p += kPartThreads) {
        const uint32_t o = tbase[sdig[p]] + p;
        if (o - seg_lo < seg_len) {
            dst_keys[o] = skeys[p];
            if (HAS_IDS || dst_ids) dst_ids[o] = sids[p];  // positions may be dropped
        }
    }
}

// ------------------------------------------------------ grouped probing ---

// Puts values computed in grouped order back in input order.  Entry e of
// partition tile t was written (HAS_IDS = false, so its id is its input
// position) to base(t, d) + its rank inside the tile's run of digit d, with
// its position in gpos.  The runs of kUngroupTiles consecutive tiles are
// adjacent in grouped order, so one workgroup takes such a group of tiles:
// its run of digit d is [base(t0, d), next(t1, d)), next being base(t1, d),
// or past the last tile the start of digit d + 1 (m after the last digit),
// long enough that every read uses whole lines.  Each thread takes entries
// of the group's runs in order (a binary search over the runs' starts gives
// the digit: skew only lengthens runs), loads position and value, places the
// value in LDS by its position, and the group's values are then written in
// input order.  One segment (S = 1).
constexpr uint32_t kUngroupThreads = 1024;
constexpr uint32_t kUngroupTiles = 4;
constexpr uint32_t kUngroupSpan = kUngroupTiles * kPartTile;  // entries per workgroup

__global__ __launch_bounds__(kUngroupThreads) void k_ungroup_by_pos(
    uint64_t m, uint32_t ntiles, uint32_t bits, const uint32_t* __restrict__ base,
    uint32_t groups, const uint32_t* __restrict__ gpos, const uint32_t* __restrict__ src,
    uint32_t* __restrict__ dst, const uint32_t* __restrict__ gate) {
    if (gate && *gate != 1u) return;  // the probe kept input order
    extern __shared__ __align__(16) uint32_t ush[];
    uint32_t* sval = ush;                          // [kUngroupSpan]
    uint32_t* rstart = sval + kUngroupSpan;        // [D + 1] run starts inside the group
    uint32_t* rbase = rstart + (1u << bits) + 1;   // [D] grouped start - run start
    uint32_t* tmp = rbase + (1u << bits);          // [kUngroupThreads / 64 + 1]
    const uint32_t D = 1u << bits;
    const uint32_t gi = xcd_tile(blockIdx.x, groups);
    if (gi >= groups) return;
    const uint32_t t0 = gi * kUngroupTiles;
    const uint32_t t1 = t0 + kUngroupTiles < ntiles ? t0 + kUngroupTiles : ntiles;
    const uint64_t begin = (uint64_t)t0 * kPartTile;
    const uint64_t end64 = (uint64_t)t1 * kPartTile;
    const uint32_t cnt = (uint32_t)((end64 < m ? end64 : m) - begin);
    constexpr uint32_t kPer = (1u << kMaxDigitBits) / kUngroupThreads;
    const uint32_t per = (D + kUngroupThreads - 1) / kUngroupThreads;
    const uint32_t d0 = threadIdx.x * per;
    const uint32_t* row = base + (size_t)t0 * D;
    const uint32_t* nrow = base + (size_t)t1 * D;
    uint32_t b[kPer], c[kPer];
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
        const uint32_t d = d0 + j;
        b[j] = c[j] = 0;
        if (j < per && d < D) {
            b[j] = row[d];
            const uint32_t nx =
                t1 < ntiles ? nrow[d] : (d + 1 < D ? base[d + 1] : (uint32_t)m);
            c[j] = nx - b[j];
        }
        mine += c[j];
    }
    uint32_t all;
    uint32_t run = block_excl_scan<kUngroupThreads>(mine, tmp, &all);
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
        const uint32_t d = d0 + j;
        if (j < per && d < D) {
            rstart[d] = run;
            rbase[d] = b[j] - run;
            run += c[j];
        }
    }
    __syncthreads();
    // all grouped positions of a thread first, then their loads, so that the
    // loads overlap
    constexpr int IT = kUngroupSpan / kUngroupThreads;
    uint32_t o[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t p = r * kUngroupThreads + threadIdx.x;
        o[r] = ~0u;
        if (p < cnt) {
            uint32_t lo = 0, hi = D;  // the last digit whose run starts at or before p
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (rstart[mid] <= p) lo = mid;
                else hi = mid;
            }
            o[r] = rbase[lo] + p;
        }
    }
    uint32_t gp[IT], v[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        gp[r] = o[r] < m ? gpos[o[r]] : 0u;
        v[r] = o[r] < m ? src[o[r]] : 0u;
    }
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint64_t li = (uint64_t)gp[r] - begin;
        if (o[r] < m && li < cnt) sval[li] = v[r];
    }
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < cnt; p += kUngroupThreads) dst[begin + p] = sval[p];
}

// A range holding more than kGroupSkew times an even share of the sampled
// queries keeps a probe in input order.
constexpr uint32_t kGroupSkew = 8;

// Whether grouping pays for these queries, from a sample: up to kGroupSample
// queries spread evenly over the input are hashed into the ranges, and when
// one range holds more than kGroupSkew times an even share of them the probe
// keeps input order (skewed queries read few index lines, which stay cached
// anyway).  Writes the one segment of the grouping passes -- with no tiles
// at all for input order, so that every grouping kernel returns at once --
// and gate[0] = 1 (grouped) or 0 (input order).  One workgroup.
constexpr uint32_t kGroupSample = 1u << 14;  // 16 per thread, loaded together

template <typename Key>
__global__ __launch_bounds__(1024) void k_group_sample(const Key* __restrict__ q, uint64_t m,
                                                       typename KeyTraits<Key>::Params hp,
                                                       uint32_t shift, uint32_t bits, Segs g,
                                                       uint32_t ntiles, uint32_t nchunks,
                                                       uint32_t* __restrict__ gate) {
    __shared__ uint32_t cnt[1u << kMaxDigitBits];
    __shared__ uint32_t wmax[1024 / kWave];
    const uint32_t D = 1u << bits;
    for (uint32_t d = threadIdx.x; d < D; d += 1024) cnt[d] = 0;
    __syncthreads();
    const uint32_t S = m < kGroupSample ? (uint32_t)m : kGroupSample;
    constexpr int IT = kGroupSample / 1024;
    Key k[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t i = r * 1024 + threadIdx.x;
        k[r] = i < S ? q[(uint64_t)i * m / S] : (Key)0;
    }
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t i = r * 1024 + threadIdx.x;
        if (i < S) atomicAdd(&cnt[(KeyTraits<Key>::bucket(k[r], hp) >> shift) & (D - 1)], 1u);
    }
    __syncthreads();
    uint32_t mx = 0;
    for (uint32_t d = threadIdx.x; d < D; d += 1024) mx = cnt[d] > mx ? cnt[d] : mx;
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t x = (uint32_t)__shfl_xor((int)mx, o, kWave);
        mx = x > mx ? x : mx;
    }
    if (lane_id() == 0) wmax[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 1024 / kWave; ++w) mx = wmax[w] > mx ? wmax[w] : mx;
        const bool grouped = (uint64_t)mx * D <= (uint64_t)kGroupSkew * S;
        gate[0] = grouped ? 1u : 0u;
        g.seg_start[0] = 0;
        g.seg_start[1] = (uint32_t)m;
        g.tile_prefix[0] = 0;
        g.tile_prefix[1] = grouped ? ntiles : 0u;
        g.chunk_prefix[0] = 0;
        g.chunk_prefix[1] = grouped ? nchunks : 0u;
    }
}

size_t ungroup_smem(uint32_t bits) {
    return 4 * ((size_t)kUngroupSpan + 2 * ((size_t)1 << bits) + 1 + kUngroupThreads / 64 + 1);
}

template <typename Key>
size_t partition_smem(uint32_t bits) {
    const size_t D = 1u << bits;
    return kPartTile * (sizeof(Key) + 4 + 2) + W_PART * D * 4 + 2 * D * 4 + (W_PART + 1) * 4 +
           64;
}

// -------------------------------------------------------- segment setup ---

// Tier-1 segment: the whole input; also clears the build's device counters
// (oversize bins, split bins, their slices, and the general key-run pass's
// two work counters).
__global__ void k_segs_single(Segs g, uint32_t n, uint32_t ntiles, uint32_t nchunks,
                              uint32_t* ctr) {
    if (threadIdx.x < 5) ctr[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        g.seg_start[0] = 0;
        g.seg_start[1] = n;
        g.tile_prefix[0] = 0;
        g.tile_prefix[1] = ntiles;
        g.chunk_prefix[0] = 0;
        g.chunk_prefix[1] = nchunks;
    }
}

// Tier-2 segments: one per tier-1 digit, from row 0 of the scanned tier-1
// matrix (the start of every digit's range).  One workgroup; S <= 2048.
__global__ __launch_bounds__(1024) void k_segs_from_bases(const uint32_t* __restrict__ base1,
                                                          uint32_t ntiles1, uint32_t n, Segs g) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
    const uint32_t S = g.S;
    const uint32_t per = (S + 1023) / 1024;  // <= 2
    uint32_t nt[2] = {0, 0}, nc[2] = {0, 0}, st[2] = {0, 0};
    uint32_t mt = 0, mc = 0;
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t a = threadIdx.x * per + j;
        if (a < S) {
            const uint32_t s0 = ntiles1 ? base1[a] : 0u;
            const uint32_t s1 = (a + 1 < S) ? (ntiles1 ? base1[a + 1] : 0u) : n;
            st[j] = s0;
            nt[j] = (s1 - s0 + kPartTile - 1) / kPartTile;
            nc[j] = (nt[j] + g.ch - 1) / g.ch;
            mt += nt[j];
            mc += nc[j];
        }
    }
    uint32_t tt, tc;
    uint32_t rt = block_excl_scan<1024>(mt, tmp, &tt);
    uint32_t rc = block_excl_scan<1024>(mc, tmp, &tc);
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t a = threadIdx.x * per + j;
        if (a < S) {
            g.seg_start[a] = st[j];
            g.tile_prefix[a] = rt;
            g.chunk_prefix[a] = rc;
            rt += nt[j];
            rc += nc[j];
        }
    }
    if (threadIdx.x == 0) {
        g.seg_start[S] = n;
        g.tile_prefix[S] = tt;
        g.chunk_prefix[S] = tc;
    }
}

// Start of every final bin (bin = segment * 2^bits + digit) in the
// partitioned array, bin_start[bins] = n, offsets[V] = n, and the list of
// bins too large for the LDS kernel.
// Bins above kSliceKeys keys are split into slices of kSliceKeys for several
// workgroups: they are listed in huge_list with their first slice in huge_s0,
// and slice_owner maps every slice back to its entry.  ctr: oversize bins,
// split bins, slices.
__global__ void k_bin_starts(const uint32_t* __restrict__ base, Segs g, uint32_t bits,
                             uint32_t light_keys,
                             uint32_t bins, uint32_t n, uint32_t V, uint32_t* __restrict__ bin_start,
                             uint32_t* __restrict__ offsets, uint32_t* __restrict__ heavy_list,
                             uint32_t* __restrict__ ctr, uint32_t* __restrict__ huge_list,
                             uint32_t* __restrict__ huge_s0, uint32_t* __restrict__ slice_owner,
                             uint32_t huge_cap, uint32_t slice_cap) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t st = 0, nx = 0;
    bool have = false;
    if (b <= bins) {
        const uint32_t D = 1u << bits;
        auto start_of = [&](uint32_t x) -> uint32_t {
            if (x >= bins) return n;
            const uint32_t s = x >> bits, d = x & (D - 1);
            const uint32_t t0 = g.tile_prefix[s];
            return (g.tile_prefix[s + 1] > t0) ? base[(size_t)t0 * D + d] : g.seg_start[s];
        };
        st = start_of(b);
        bin_start[b] = st;
        if (b == bins) offsets[V] = n;
        if (b < bins) {
            nx = start_of(b + 1);
            have = nx - st > light_keys;
        }
    }
    if (have) {
        const uint32_t L = nx - st;
        if (L <= kSliceKeys) {
            const uint32_t slot = atomicAdd(&ctr[0], 1u);
            heavy_list[slot] = b;
        } else {
            // capacities hold: a split bin has > kSliceKeys keys, so there are
            // at most n / kSliceKeys of them and fewer than 2n / kSliceKeys slices
            const uint32_t ns = (L + kSliceKeys - 1) / kSliceKeys;
            const uint32_t idx = atomicAdd(&ctr[1], 1u);
            const uint32_t s0 = atomicAdd(&ctr[2], ns);
            if (idx < huge_cap && s0 + ns <= slice_cap) {
                huge_list[idx] = b;
                huge_s0[idx] = s0;
                for (uint32_t j = 0; j < ns; ++j) slice_owner[s0 + j] = idx;
            }
        }
    }
}

// Slice `item` of a split bin: its bin and key range.
struct SliceRef {
    uint32_t idx, b, begin, end;
};

__device__ __forceinline__ SliceRef slice_at(uint32_t item, const uint32_t* __restrict__ bin_start,
                                             const uint32_t* __restrict__ huge_list,
                                             const uint32_t* __restrict__ huge_s0,
                                             const uint32_t* __restrict__ slice_owner) {
    SliceRef r;
    r.idx = slice_owner[item];
    r.b = huge_list[r.idx];
    const uint32_t j = item - huge_s0[r.idx];
    const uint32_t bs = bin_start[r.b], be = bin_start[r.b + 1];
    r.begin = bs + j * kSliceKeys;
    r.end = (be - r.begin > kSliceKeys) ? r.begin + kSliceKeys : be;
    return r;
}

// Per-slice bucket histograms of the split bins: hist[item][0 .. 2^k).
template <typename Key>
__global__ __launch_bounds__(kLocalThreads) void k_huge_hist(
    const Key* __restrict__ src_keys, const uint32_t* __restrict__ bin_start,
    const uint32_t* __restrict__ huge_list, const uint32_t* __restrict__ huge_s0,
    const uint32_t* __restrict__ slice_owner, const uint32_t* __restrict__ ctr,
    typename KeyTraits<Key>::Params hp, uint32_t k, uint32_t* __restrict__ hist) {
    extern __shared__ uint32_t cnt[];
    const uint32_t NB = 1u << k, nsl = ctr[2];
    for (uint32_t item = blockIdx.x; item < nsl; item += gridDim.x) {
        const SliceRef r = slice_at(item, bin_start, huge_list, huge_s0, slice_owner);
        const uint32_t v0 = r.b << k;
        for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads) cnt[i] = 0;
        __syncthreads();
        // a split bin holds a hot key: lanes sharing the first active lane's
        // bucket add their count with one LDS atomic, the others one each
        for (uint32_t i = r.begin + threadIdx.x; i < r.end; i += kLocalThreads) {
            const uint32_t b = KeyTraits<Key>::bucket(src_keys[i], hp) - v0;
            const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b);
            const uint64_t same = ballot(b == b0);
            if (b != b0) atomicAdd(&cnt[b], 1u);
            else if (mbcnt(same) == 0) atomicAdd(&cnt[b0], (uint32_t)__popcll(same));
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads)
            hist[(size_t)item * NB + i] = cnt[i];
        __syncthreads();
    }
}

// The scan over the split bins' slice histograms, in three steps so that a
// bin of many slices is spread over many threads: per (bin, bucket) the total
// over the bin's slices; per bin the bucket starts (written to offsets, and
// kept in place of the totals); per (bin, bucket) the position of every
// slice's first entry of the bucket, in place of its count.

// Slices of split bin idx: [s0, s0 + ns).
__device__ __forceinline__ uint32_t huge_slices(const uint32_t* __restrict__ bin_start,
                                                const uint32_t* __restrict__ huge_list,
                                                uint32_t idx) {
    const uint32_t b = huge_list[idx];
    return (bin_start[b + 1] - bin_start[b] + kSliceKeys - 1) / kSliceKeys;
}

__global__ __launch_bounds__(256) void k_huge_tot(
    const uint32_t* __restrict__ bin_start, const uint32_t* __restrict__ huge_list,
    const uint32_t* __restrict__ huge_s0, const uint32_t* __restrict__ ctr, uint32_t k,
    uint32_t huge_cap, const uint32_t* __restrict__ hist, uint32_t* __restrict__ tot) {
    const uint32_t NB = 1u << k, nh = ctr[1] < huge_cap ? ctr[1] : huge_cap;
    const uint64_t all = (uint64_t)nh << k, st = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < all; x += st) {
        const uint32_t idx = (uint32_t)(x >> k), v = (uint32_t)x & (NB - 1);
        const uint32_t s0 = huge_s0[idx], ns = huge_slices(bin_start, huge_list, idx);
        const uint32_t* h = hist + (size_t)s0 * NB + v;
        uint32_t acc = 0;
#pragma unroll 4
        for (uint32_t sl = 0; sl < ns; ++sl) acc += h[(size_t)sl * NB];
        tot[x] = acc;
    }
}

__global__ __launch_bounds__(kLocalThreads) void k_huge_starts(
    const uint32_t* __restrict__ bin_start, const uint32_t* __restrict__ huge_list,
    const uint32_t* __restrict__ ctr, uint32_t k, uint32_t V, uint32_t huge_cap,
    uint32_t* __restrict__ tot, uint32_t* __restrict__ offsets) {
    __shared__ uint32_t tmp[kLocalThreads / kWave + 1];
    const uint32_t NB = 1u << k, nh = ctr[1] < huge_cap ? ctr[1] : huge_cap;
    const uint32_t per = NB >= (uint32_t)kLocalThreads ? NB / kLocalThreads : 1u;  // <= 16
    const uint32_t i0 = threadIdx.x * per;
    for (uint32_t idx = blockIdx.x; idx < nh; idx += gridDim.x) {
        const uint32_t b = huge_list[idx];
        const uint32_t v0 = b << k, nb = (V - v0 < NB) ? V - v0 : NB;
        uint32_t* t = tot + ((size_t)idx << k);
        uint32_t c[16];
        uint32_t mine = 0;
        for (uint32_t j = 0; j < per; ++j) {
            c[j] = i0 + j < NB ? t[i0 + j] : 0u;
            mine += c[j];
        }
        uint32_t all;
        uint32_t run = bin_start[b] + block_excl_scan<kLocalThreads>(mine, tmp, &all);
        for (uint32_t j = 0; j < per; ++j) {
            const uint32_t v = i0 + j;
            if (v < NB) {
                if (v < nb) offsets[v0 + v] = run;
                t[v] = run;
            }
            run += c[j];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_huge_down(
    const uint32_t* __restrict__ bin_start, const uint32_t* __restrict__ huge_list,
    const uint32_t* __restrict__ huge_s0, const uint32_t* __restrict__ ctr, uint32_t k,
    uint32_t huge_cap, const uint32_t* __restrict__ tot, uint32_t* __restrict__ hist) {
    const uint32_t NB = 1u << k, nh = ctr[1] < huge_cap ? ctr[1] : huge_cap;
    const uint64_t all = (uint64_t)nh << k, st = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < all; x += st) {
        const uint32_t idx = (uint32_t)(x >> k), v = (uint32_t)x & (NB - 1);
        const uint32_t s0 = huge_s0[idx], ns = huge_slices(bin_start, huge_list, idx);
        uint32_t* h = hist + (size_t)s0 * NB + v;
        uint32_t r = tot[x];
        for (uint32_t sl = 0; sl < ns; ++sl) {
            const uint32_t c = h[(size_t)sl * NB];
            h[(size_t)sl * NB] = r;
            r += c;
        }
    }
}

// Stable placement of every slice of the split bins, from its cursors.
template <typename Key>
__global__ __launch_bounds__(kLocalThreads) void k_huge_place(
    const Key* __restrict__ src_keys, const uint32_t* __restrict__ src_ids,
    const uint32_t* __restrict__ bin_start, const uint32_t* __restrict__ huge_list,
    const uint32_t* __restrict__ huge_s0, const uint32_t* __restrict__ slice_owner,
    const uint32_t* __restrict__ ctr, typename KeyTraits<Key>::Params hp, uint32_t k,
    const uint32_t* __restrict__ hist, uint32_t* __restrict__ ids, Key* __restrict__ ekeys,
    bool any_order) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t NB = 1u << k, nsl = ctr[2];
    const HeavyLds<Key> m(smem, NB);
    for (uint32_t item = blockIdx.x; item < nsl; item += gridDim.x) {
        const SliceRef r = slice_at(item, bin_start, huge_list, huge_s0, slice_owner);
        for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads)
            m.cur[i] = hist[(size_t)item * NB + i];
        __syncthreads();
        place_in_chunks<Key>(src_keys + r.begin, src_ids + r.begin, 0u, r.end - r.begin,
                             bin_start[r.b], bin_start[r.b + 1], r.b << k, k, hp, ids, ekeys,
                             smem, any_order);
        __syncthreads();
    }
}

// Probe index entries of the split bins' buckets (after their placement);
// their long buckets are listed for the general pass of the key runs.
template <typename Key>
__global__ __launch_bounds__(kLocalThreads) void k_huge_index(
    const uint32_t* __restrict__ bin_start, const uint32_t* __restrict__ huge_list,
    const uint32_t* __restrict__ ctr, uint32_t k, uint32_t V,
    const uint32_t* __restrict__ offsets, const Key* __restrict__ ekeys, IndexOut ix) {
    __shared__ uint32_t nlisted;
    const uint32_t NB = 1u << k, nh = ctr[1];
    for (uint32_t idx = blockIdx.x; idx < nh; idx += gridDim.x) {
        const uint32_t b = huge_list[idx];
        const uint32_t v0 = b << k, nb = (V - v0 < NB) ? V - v0 : NB;
        const uint32_t bs = bin_start[b], be = bin_start[b + 1];
        if (threadIdx.x == 0) nlisted = 0;
        __syncthreads();
        for (uint32_t v = threadIdx.x; v < nb; v += kLocalThreads) {
            const uint32_t lo = offsets[v0 + v];
            const uint32_t hi = (v + 1 < nb) ? offsets[v0 + v + 1] : be;
            if (hi - lo > kRunBucket)
                ix.gen_list[gen_region(bs, b) + atomicAdd(&nlisted, 1u)] = v0 + v;
            else
                ix.head[v0 + v] = head_entry<Key>(lo, hi, ekeys + lo);
        }
        __syncthreads();
        if (threadIdx.x == 0) ix.gen_cnt[b] = nlisted;
        __syncthreads();
    }
}

// One workgroup per final bin g (buckets [g*2^k, min((g+1)*2^k, V))) that
// holds at most light_cap<Key>() keys.
template <typename Key>
__global__ __launch_bounds__(kLocalThreads) void k_local_light(
    const Key* __restrict__ src_keys, const uint32_t* __restrict__ src_ids,
    const uint32_t* __restrict__ bin_start, typename KeyTraits<Key>::Params hp, uint32_t k,
    uint32_t* __restrict__ offsets, IndexOut ix, uint32_t* __restrict__ ids,
    Key* __restrict__ ekeys, bool any_order) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t g = blockIdx.x;
    const uint32_t start = bin_start[g], end = bin_start[g + 1];
    const uint32_t L = end - start;
    if (L > light_cap<Key>()) return;  // oversize bins go to k_local_heavy
    const uint32_t NB = 1u << k, v0 = g << k, V = hp.range;
    const uint32_t nb = (V - v0 < NB) ? V - v0 : NB;
    light_bin_body<Key>(src_keys + start, src_ids + start, 0u, L, start, v0, k, nb, hp, offsets,
                        ix, ids, ekeys, smem, any_order);
}

// Oversize bins (from the device list), one workgroup per bin.
template <typename Key>
__global__ __launch_bounds__(kLocalThreads) void k_local_heavy(
    const Key* __restrict__ src_keys, const uint32_t* __restrict__ src_ids,
    const uint32_t* __restrict__ bin_start, const uint32_t* __restrict__ heavy_list,
    const uint32_t* __restrict__ heavy_count, typename KeyTraits<Key>::Params hp, uint32_t k,
    uint32_t* __restrict__ offsets, IndexOut ix, uint32_t* __restrict__ ids,
    Key* __restrict__ ekeys, bool any_order) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t NB = 1u << k, V = hp.range;
    const uint32_t nheavy = *heavy_count;
    for (uint32_t i = blockIdx.x; i < nheavy; i += gridDim.x) {
        const uint32_t g = heavy_list[i];
        const uint32_t start = bin_start[g], end = bin_start[g + 1];
        const uint32_t v0 = g << k;
        const uint32_t nb = (V - v0 < NB) ? V - v0 : NB;
        heavy_bin_body<Key>(src_keys + start, src_ids + start, 0u, end - start, start, v0, k, nb,
                            hp, offsets, ix, ids, ekeys, smem, any_order);
        __syncthreads();
    }
}

// Final step of the scatter by a permutation: bin g holds the entries whose
// ids are [g << k, (g << k) + 2^k) (every id occurs once, so the bin starts at
// g << k after the partition passes); they are placed in LDS by id and
// written out with coalesced stores.
__global__ __launch_bounds__(512) void k_perm_place(const uint32_t* __restrict__ vals,
                                                    const uint32_t* __restrict__ ids, uint64_t n,
                                                    uint32_t k, uint32_t* __restrict__ out) {
    __shared__ uint32_t buf[1u << kMaxLocalBits];
    const uint64_t start = (uint64_t)blockIdx.x << k;
    const uint32_t len = (uint32_t)(n - start < (1ull << k) ? n - start : (1ull << k));
    for (uint32_t i = threadIdx.x; i < len; i += 512) {
        const uint32_t off = (uint32_t)(ids[start + i] - start);
        if (off < len) buf[off] = vals[start + i];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < len; i += 512) out[start + i] = buf[i];
}

__global__ void k_perm_direct(const uint32_t* __restrict__ ids, const uint32_t* __restrict__ vals,
                              uint64_t n, uint32_t* __restrict__ out) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (; p < n; p += st) {
        const uint32_t id = ids[p];
        if (id < n) out[id] = vals[p];
    }
}

constexpr uint64_t kPermDirectMax = 1ull << 20;  // below this the output stays in L2

V2Plan perm_plan(uint64_t n);

}  // namespace

// ------------------------------------------------------------------ plan --

V2Plan plan_v2(uint64_t n, uint64_t V, int key_bits, uint32_t bins_hint) {
    V2Plan p;
    p.n = n;
    p.V = V;
    uint32_t k;
    if (bins_hint) {
        k = log2_ceil(ceil_div(V, bins_hint));
    } else if (n == 0) {
        k = kMaxLocalBits;
    } else {
        // about 4096 keys per final bin for 32-bit keys (2^k * n / V ~ 4096),
        // 2048 for 64-bit keys, whose LDS bin then still leaves room for two
        // workgroups per CU
        const double target = key_bits == 64 ? 2048.0 : 4096.0;
        const double r = target * (double)V / (double)n;
        k = 0;
        while (k < kMaxLocalBits && (double)(1ull << (k + 1)) <= r) ++k;
    }
    if (k > kMaxLocalBits) k = kMaxLocalBits;
    const uint32_t kv = log2_ceil(V);
    if (k > kv) k = kv;
    p.k = k;
    p.bins = (uint32_t)ceil_div(V, 1ull << k);
    const uint32_t bits = log2_ceil(p.bins);
    if (bits <= kOneTierBits) {
        p.tiers = 1;
        p.b1 = bits;
        p.b2 = 0;
    } else {
        p.tiers = 2;
        p.b1 = bits / 2;
        p.b2 = bits - p.b1;
    }
    p.ntiles1 = (uint32_t)ceil_div(n, kPartTile);
    p.ch1 = (uint32_t)pow2_ceil(ceil_div(p.ntiles1 ? p.ntiles1 : 1, 256));
    p.nchunks1 = (uint32_t)ceil_div(p.ntiles1, p.ch1);
    if (p.tiers == 2) {
        const uint32_t S = 1u << p.b1;
        p.ntiles2_ub = p.ntiles1 + S;
        p.ch2 = (uint32_t)pow2_ceil(ceil_div(p.ntiles1 ? p.ntiles1 : 1, (uint64_t)S * 4));
        p.nchunks2_ub = (uint32_t)ceil_div(p.ntiles2_ub, p.ch2) + S;
    }
    return p;
}

namespace {

struct V2Ws {
    void* rkeys;
    uint32_t* rids;
    uint32_t *m1, *c1, *m2, *c2, *bin_start, *heavy_list;
    uint32_t* ctr;  // [5]: oversize bins, split bins, slices of split bins, key-run work
    uint32_t *huge_list, *huge_s0, *slice_owner, *slice_hist, *huge_tot;
    uint32_t huge_cap, slice_cap;
    uint32_t *gen_list, *gen_cnt;  // long buckets left to the general key-run pass
    void* runs_ws;
    Segs s1, s2;
};

// One layout used both to size the workspace (base == nullptr) and to carve it.
size_t layout_v2(void* ws, const V2Plan& p, size_t key_size, V2Ws* out) {
    Carver c(ws);
    V2Ws w{};
    w.rkeys = c.take<char>(p.n * key_size);
    w.rids = c.take<uint32_t>(p.n);
    const uint32_t D1 = 1u << p.b1, D2 = 1u << p.b2;
    w.m1 = c.take<uint32_t>((size_t)p.ntiles1 * D1);
    w.c1 = c.take<uint32_t>((size_t)p.nchunks1 * D1);
    w.s1.seg_start = c.take<uint32_t>(2);
    w.s1.tile_prefix = c.take<uint32_t>(2);
    w.s1.chunk_prefix = c.take<uint32_t>(2);
    w.s1.S = 1;
    w.s1.ch = p.ch1;
    if (p.tiers == 2) {
        w.m2 = c.take<uint32_t>((size_t)p.ntiles2_ub * D2);
        w.c2 = c.take<uint32_t>((size_t)p.nchunks2_ub * D2);
        w.s2.seg_start = c.take<uint32_t>(D1 + 1);
        w.s2.tile_prefix = c.take<uint32_t>(D1 + 1);
        w.s2.chunk_prefix = c.take<uint32_t>(D1 + 1);
        w.s2.S = D1;
        w.s2.ch = p.ch2;
    }
    w.bin_start = c.take<uint32_t>((size_t)p.bins + 1);
    w.heavy_list = c.take<uint32_t>((size_t)p.bins);
    w.ctr = c.take<uint32_t>(5);
    w.huge_cap = (uint32_t)(p.n / kSliceKeys + 1);
    w.slice_cap = 2 * w.huge_cap;
    w.huge_list = c.take<uint32_t>(w.huge_cap);
    w.huge_s0 = c.take<uint32_t>(w.huge_cap);
    w.slice_owner = c.take<uint32_t>(w.slice_cap);
    w.slice_hist = c.take<uint32_t>((size_t)w.slice_cap << p.k);
    w.huge_tot = c.take<uint32_t>((size_t)w.huge_cap << p.k);
    w.gen_list = c.take<uint32_t>(gen_list_cap(p.n, p.bins));
    w.gen_cnt = c.take<uint32_t>((size_t)p.bins + 1);
    w.runs_ws = c.take<char>(runs_ws_bytes(p.n, p.bins));
    if (out) *out = w;
    return c.off + 256;
}

// for_probe: profiled under the grouped probe's names
hipError_t colscan(uint32_t* mat, const Segs& g, uint32_t D, uint32_t* csum, uint32_t nchunks_ub,
                   hipStream_t s, bool for_probe) {
    {
        HG_PROF(for_probe ? "probe_group_scan_reduce" : "v2_colscan_reduce", s);
        hipLaunchKernelGGL(k_colscan_reduce, dim3(nchunks_ub), dim3(256), 0, s,
                           (const uint32_t*)mat, g, D, csum);
    }
    HG_TRY(hipGetLastError());
    {
        HG_PROF(for_probe ? "probe_group_scan_seg" : "v2_colscan_seg", s);
        hipLaunchKernelGGL(k_colscan_seg, dim3(g.S), dim3(256), 0, s, g, D, csum);
    }
    HG_TRY(hipGetLastError());
    {
        HG_PROF(for_probe ? "probe_group_scan_down" : "v2_colscan_down", s);
        hipLaunchKernelGGL(k_colscan_down, dim3(nchunks_ub), dim3(256), 0, s, mat, g, D,
                           (const uint32_t*)csum);
    }
    return hipGetLastError();
}

template <typename Key, bool HAS_IDS, bool STABLE>
void launch_partition(dim3 grid, size_t smem, hipStream_t s, const Key* src_keys,
                      const uint32_t* src_ids, Key* dst_keys, uint32_t* dst_ids, const Segs& g,
                      typename KeyTraits<Key>::Params hp, uint32_t shift, uint32_t bits,
                      const uint32_t* mat, uint32_t tiles_ub) {
    hipLaunchKernelGGL((k_tile_partition<Key, HAS_IDS, STABLE>), grid, dim3(kPartThreads), smem,
                       s, src_keys, src_ids, dst_keys, dst_ids, g, hp, shift, bits, mat,
                       tiles_ub);
}

// One stable (or any-order) partition pass over the tiles of segments g.
// id_digit (32-bit entries with ids only): the digit comes from the id.
// tier: 1 or 2 for the build's passes, 3 for grouping the queries of a probe
// (profiled under its own names); dst_ids may be null without src_ids.
template <typename Key>
hipError_t partition_pass(const Key* src_keys, const uint32_t* src_ids, Key* dst_keys,
                          uint32_t* dst_ids, const Segs& g, typename KeyTraits<Key>::Params hp,
                          uint32_t shift, uint32_t bits, uint32_t* mat, uint32_t* csum,
                          uint32_t tiles_ub, uint32_t nchunks_ub, int tier, bool stable,
                          hipStream_t s, bool id_digit = false) {
    const uint32_t D = 1u << bits;
    const uint32_t grid = (uint32_t)(8 * ceil_div(tiles_ub, 8));
    if (id_digit && (sizeof(Key) != 4 || !src_ids || stable)) return hipErrorInvalidValue;
    if (bits > kMaxDigitBits) return hipErrorInvalidValue;  // the kernels hold at most 2048 digits
    {
        HG_PROF(tier == 1 ? "v2_tile_hist_t1" : tier == 2 ? "v2_tile_hist_t2" : "probe_group_hist", s);
        if (id_digit)
            hipLaunchKernelGGL((k_tile_hist<Key, true>), dim3(grid), dim3(kPartThreads), D * 4, s,
                               src_keys, g, hp, shift, bits, mat, tiles_ub, src_ids);
        else if (tier == 3)
            hipLaunchKernelGGL((k_tile_hist<Key, false, true>), dim3(grid), dim3(kPartThreads),
                               D * 4, s, src_keys, g, hp, shift, bits, mat, tiles_ub, nullptr);
        else
            hipLaunchKernelGGL((k_tile_hist<Key, false>), dim3(grid), dim3(kPartThreads), D * 4, s,
                               src_keys, g, hp, shift, bits, mat, tiles_ub, nullptr);
    }
    HG_TRY(hipGetLastError());
    HG_TRY(colscan(mat, g, D, csum, nchunks_ub, s, tier == 3));
    const size_t smem = partition_smem<Key>(bits);
    {
        HG_PROF(tier == 1 ? "v2_partition_t1" : tier == 2 ? "v2_partition_t2" : "probe_group", s);
        const dim3 gr(grid);
        if (id_digit)
            hipLaunchKernelGGL((k_tile_partition<Key, true, false, true>), gr, dim3(kPartThreads),
                               smem, s, src_keys, src_ids, dst_keys, dst_ids, g, hp, shift, bits,
                               (const uint32_t*)mat, tiles_ub);
        else if (tier == 3 && !src_ids && !stable)
            hipLaunchKernelGGL((k_tile_partition<Key, false, false, false, true>), gr,
                               dim3(kPartThreads), smem, s, src_keys, src_ids, dst_keys, dst_ids,
                               g, hp, shift, bits, (const uint32_t*)mat, tiles_ub);
        else if (src_ids && stable)
            launch_partition<Key, true, true>(gr, smem, s, src_keys, src_ids, dst_keys, dst_ids,
                                              g, hp, shift, bits, mat, tiles_ub);
        else if (src_ids)
            launch_partition<Key, true, false>(gr, smem, s, src_keys, src_ids, dst_keys, dst_ids,
                                               g, hp, shift, bits, mat, tiles_ub);
        else if (stable)
            launch_partition<Key, false, true>(gr, smem, s, src_keys, src_ids, dst_keys, dst_ids,
                                               g, hp, shift, bits, mat, tiles_ub);
        else
            launch_partition<Key, false, false>(gr, smem, s, src_keys, src_ids, dst_keys,
                                                dst_ids, g, hp, shift, bits, mat, tiles_ub);
    }
    return hipGetLastError();
}

template <typename Key>
hipError_t set_smem_limits() {
    static std::atomic<uint64_t> done{0};
    return once_per_device(done, [] {
        const int lim = 160 * 1024;
        HG_TRY(hipFuncSetAttribute((const void*)k_tile_partition<Key, true, true>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_tile_partition<Key, false, true>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_tile_partition<Key, true, false>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_tile_partition<Key, true, false, true>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_tile_partition<Key, false, false>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_tile_partition<Key, false, false, false, true>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_local_light<Key>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_local_heavy<Key>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_huge_place<Key>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        HG_TRY(hipFuncSetAttribute((const void*)k_ungroup_by_pos,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        return hipSuccess;
    });
}

}  // namespace

size_t build_ws_bytes(int variant, uint64_t n, uint64_t V, int key_bits, uint32_t bins_hint) {
    const size_t ks = key_bits == 64 ? 8 : 4;
    if (variant == 1) {
        Carver c(nullptr);
        c.take<uint32_t>(V);
        c.take<char>(scan_ws_bytes(V));
        return c.off + 256;
    }
    return layout_v2(nullptr, plan_v2(n, V, key_bits, bins_hint), ks, nullptr);
}

template <typename Key>
hipError_t run_build_v2(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* offsets,
                        uint32_t* ids, Key* ekeys, IndexOut& ix, void* ws,
                        uint32_t bins_hint, bool stable, hipStream_t s) {
    HG_TRY(set_smem_limits<Key>());
    ix.k = 0;
    ix.bins = 0;
    if (n == 0) {
        if (ix.head) HG_TRY(fill_u32((uint32_t*)ix.head, 4 * V, 0u, s));
        return fill_u32(offsets, V + 1, 0u, s);
    }
    const V2Plan p = plan_v2(n, V, sizeof(Key) * 8, bins_hint);
    ix.k = p.k;
    ix.bins = p.bins;
    V2Ws w;
    layout_v2(ws, p, sizeof(Key), &w);
    ix.gen_list = w.gen_list;
    ix.gen_cnt = w.gen_cnt;
    auto hp = KeyTraits<Key>::make(V, seed);
    Key* rkeys = (Key*)w.rkeys;
    {
        HG_PROF("v2_segs", s);
        hipLaunchKernelGGL(k_segs_single, dim3(1), dim3(64), 0, s, w.s1, (uint32_t)n, p.ntiles1,
                           p.nchunks1, w.ctr);
    }
    HG_TRY(hipGetLastError());
    const uint32_t* bin_mat;
    Segs bin_segs;
    uint32_t bin_bits;
    if (p.tiers == 1) {
        HG_TRY(partition_pass<Key>(keys, nullptr, rkeys, w.rids, w.s1, hp, p.k, p.b1, w.m1, w.c1,
                                   p.ntiles1, p.nchunks1, 1, stable, s));
        bin_mat = w.m1;
        bin_segs = w.s1;
        bin_bits = p.b1;
    } else {
        // tier 1 into the table's own arrays, tier 2 into the workspace
        HG_TRY(partition_pass<Key>(keys, nullptr, ekeys, ids, w.s1, hp, p.k + p.b2, p.b1, w.m1,
                                   w.c1, p.ntiles1, p.nchunks1, 1, stable, s));
        {
            HG_PROF("v2_segs", s);
            hipLaunchKernelGGL(k_segs_from_bases, dim3(1), dim3(1024), 0, s,
                               (const uint32_t*)w.m1, p.ntiles1, (uint32_t)n, w.s2);
        }
        HG_TRY(hipGetLastError());
        HG_TRY(partition_pass<Key>(ekeys, ids, rkeys, w.rids, w.s2, hp, p.k, p.b2, w.m2, w.c2,
                                   p.ntiles2_ub, p.nchunks2_ub, 2, stable, s));
        bin_mat = w.m2;
        bin_segs = w.s2;
        bin_bits = p.b2;
    }
    {
        HG_PROF("v2_bin_starts", s);
        hipLaunchKernelGGL(k_bin_starts, dim3((uint32_t)ceil_div(p.bins + 1, 256)), dim3(256), 0,
                           s, bin_mat, bin_segs, bin_bits, light_cap<Key>(), p.bins, (uint32_t)n,
                           (uint32_t)V,
                           w.bin_start, offsets, w.heavy_list, w.ctr, w.huge_list, w.huge_s0,
                           w.slice_owner, w.huge_cap, w.slice_cap);
    }
    HG_TRY(hipGetLastError());
    {
        HG_PROF("v2_local_build", s);
        hipLaunchKernelGGL(k_local_light<Key>, dim3(p.bins), dim3(kLocalThreads),
                           ix.head ? light_smem_index<Key>(p.k) : light_smem<Key>(p.k), s,
                           (const Key*)rkeys, (const uint32_t*)w.rids,
                           (const uint32_t*)w.bin_start, hp, p.k, offsets, ix, ids, ekeys,
                           !stable);
    }
    HG_TRY(hipGetLastError());
    {
        HG_PROF("v2_local_heavy", s);
        const uint32_t hg_grid = p.bins < 512 ? p.bins : 512;
        hipLaunchKernelGGL(k_local_heavy<Key>, dim3(hg_grid), dim3(kLocalThreads),
                           heavy_smem<Key>(p.k), s, (const Key*)rkeys, (const uint32_t*)w.rids,
                           (const uint32_t*)w.bin_start, (const uint32_t*)w.heavy_list,
                           (const uint32_t*)w.ctr, hp, p.k, offsets, ix, ids, ekeys, !stable);
    }
    HG_TRY(hipGetLastError());
    if (n > kSliceKeys) {
        // bins above kSliceKeys keys (skew): per-slice counts, per-bin scan,
        // per-slice placement; the grids drain device-side work lists
        HG_PROF("v2_split_bins", s);
        const uint32_t* bs = w.bin_start;
        hipLaunchKernelGGL(k_huge_hist<Key>, dim3(1024), dim3(kLocalThreads),
                           (size_t)4 << p.k, s, (const Key*)rkeys, bs,
                           (const uint32_t*)w.huge_list, (const uint32_t*)w.huge_s0,
                           (const uint32_t*)w.slice_owner, (const uint32_t*)w.ctr, hp, p.k,
                           w.slice_hist);
        HG_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_huge_tot, dim3(1024), dim3(256), 0, s, bs,
                           (const uint32_t*)w.huge_list, (const uint32_t*)w.huge_s0,
                           (const uint32_t*)w.ctr, p.k, w.huge_cap,
                           (const uint32_t*)w.slice_hist, w.huge_tot);
        HG_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_huge_starts, dim3(256), dim3(kLocalThreads), 0, s, bs,
                           (const uint32_t*)w.huge_list, (const uint32_t*)w.ctr, p.k,
                           (uint32_t)V, w.huge_cap, w.huge_tot, offsets);
        HG_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_huge_down, dim3(1024), dim3(256), 0, s, bs,
                           (const uint32_t*)w.huge_list, (const uint32_t*)w.huge_s0,
                           (const uint32_t*)w.ctr, p.k, w.huge_cap,
                           (const uint32_t*)w.huge_tot, w.slice_hist);
        HG_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_huge_place<Key>, dim3(1024), dim3(kLocalThreads),
                           heavy_smem<Key>(p.k), s, (const Key*)rkeys, (const uint32_t*)w.rids,
                           bs, (const uint32_t*)w.huge_list, (const uint32_t*)w.huge_s0,
                           (const uint32_t*)w.slice_owner, (const uint32_t*)w.ctr, hp, p.k,
                           (const uint32_t*)w.slice_hist, ids, ekeys, !stable);
        HG_TRY(hipGetLastError());
        if (ix.head) {
            hipLaunchKernelGGL(k_huge_index<Key>, dim3(256), dim3(kLocalThreads), 0, s, bs,
                               (const uint32_t*)w.huge_list, (const uint32_t*)w.ctr, p.k,
                               (uint32_t)V, (const uint32_t*)offsets, (const Key*)ekeys, ix);
            HG_TRY(hipGetLastError());
        }
    }
    if (ix.head)
        HG_TRY(run_key_runs<Key>(offsets, ids, ekeys, n, w.bin_start, p.bins, ix, rkeys, w.rids,
                                 w.ctr + 3, w.runs_ws, s));
    return hipSuccess;
}

// ------------------------------------------------ scatter by a permutation --
//
// out[ids[p]] = vals[p] for p < n, where ids holds every index of [0, n)
// once (a table's edge ids): Alg. 3's counts, found in B's edge order, put
// back in B's input order.  One random 4-byte store per entry would leave
// partial lines beyond the L2; instead the (value, id) pairs go through the
// same stable partition passes as a V2 build, with the digits taken from the
// id instead of a key's bucket, down to bins of 4096 consecutive ids, and
// each bin is placed in LDS and written out with coalesced stores.

namespace {

V2Plan perm_plan(uint64_t n) {
    // the ids are the "buckets": V = n, bins of 2^12 ids
    return plan_v2(n, n, 32, (uint32_t)ceil_div(n, 1ull << kMaxLocalBits));
}

size_t perm_layout(void* ws, const V2Plan& p, V2Ws* w, uint32_t** xv, uint32_t** xi) {
    Carver c(ws);
    void* v2 = c.take<char>(layout_v2(nullptr, p, 4, nullptr));
    *xv = c.take<uint32_t>(p.n);
    *xi = c.take<uint32_t>(p.n);
    if (ws) layout_v2(v2, p, 4, w);
    return c.off + 256;
}

}  // namespace

size_t scatter_perm_ws_bytes(uint64_t n) {
    if (n <= kPermDirectMax) return 256;
    uint32_t *xv, *xi;
    return perm_layout(nullptr, perm_plan(n), nullptr, &xv, &xi);
}

hipError_t scatter_perm(const uint32_t* ids, const uint32_t* vals, uint64_t n, uint32_t* out,
                        void* ws, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (n <= kPermDirectMax) {
        HG_PROF("scatter_direct", s);
        const uint64_t g = ceil_div(n, 256 * 4);
        hipLaunchKernelGGL(k_perm_direct, dim3((uint32_t)(g > 4096 ? 4096 : g)), dim3(256), 0, s,
                           ids, vals, n, out);
        return hipGetLastError();
    }
    HG_TRY(set_smem_limits<uint32_t>());
    const V2Plan p = perm_plan(n);
    V2Ws w;
    uint32_t *xv, *xi;
    perm_layout(ws, p, &w, &xv, &xi);
    const auto hp = KeyTraits<uint32_t>::make(1, 0);  // unused: digits come from the ids
    uint32_t* rv = (uint32_t*)w.rkeys;
    hipLaunchKernelGGL(k_segs_single, dim3(1), dim3(64), 0, s, w.s1, (uint32_t)n, p.ntiles1,
                       p.nchunks1, w.ctr);
    HG_TRY(hipGetLastError());
    if (p.tiers == 1) {
        HG_TRY(partition_pass<uint32_t>(vals, ids, rv, w.rids, w.s1, hp, p.k, p.b1, w.m1, w.c1,
                                        p.ntiles1, p.nchunks1, 1, false, s, true));
    } else {
        HG_TRY(partition_pass<uint32_t>(vals, ids, xv, xi, w.s1, hp, p.k + p.b2, p.b1, w.m1,
                                        w.c1, p.ntiles1, p.nchunks1, 1, false, s, true));
        hipLaunchKernelGGL(k_segs_from_bases, dim3(1), dim3(1024), 0, s, (const uint32_t*)w.m1,
                           p.ntiles1, (uint32_t)n, w.s2);
        HG_TRY(hipGetLastError());
        HG_TRY(partition_pass<uint32_t>(xv, xi, rv, w.rids, w.s2, hp, p.k, p.b2, w.m2, w.c2,
                                        p.ntiles2_ub, p.nchunks2_ub, 2, false, s, true));
    }
    {
        HG_PROF("scatter_place", s);
        hipLaunchKernelGGL(k_perm_place, dim3(p.bins), dim3(512), 0, s, (const uint32_t*)rv,
                           (const uint32_t*)w.rids, n, p.k, out);
    }
    return hipGetLastError();
}

// --------------------------------------------- grouped Probe-Standard ---
// The queries are first partitioned into up to 2^kGroupBits ranges of
// buckets with their input positions (one tile-histogram, column-scan and
// partition pass, as in the build), probed in that order with the tiles
// dealt out per XCD -- each XCD then reads one window of the index at a time
// (8 MiB at 2^28 buckets), which its L2 holds, instead of random lines of
// the whole index -- and the counts are put back in input order by
// k_ungroup_by_pos.

namespace {

constexpr uint32_t kGroupBits = 9;

struct GroupPlan {
    uint32_t bits, shift, ntiles, ch, nchunks;
};

GroupPlan group_plan(uint64_t m, uint64_t V) {
    GroupPlan p;
    const uint32_t kv = log2_ceil(V);
    p.bits = kv < kGroupBits ? (kv ? kv : 1u) : kGroupBits;  // at least two ranges
    p.shift = kv > p.bits ? kv - p.bits : 0u;
    p.ntiles = (uint32_t)ceil_div(m, kPartTile);
    p.ch = (uint32_t)pow2_ceil(ceil_div(p.ntiles ? p.ntiles : 1, 256));
    p.nchunks = (uint32_t)ceil_div(p.ntiles, p.ch);
    return p;
}

struct GroupWs {
    void* gq;        // the queries in grouped order
    uint32_t* gpos;  // their input positions
    uint32_t* gc;    // their counts in grouped order
    uint32_t *mat, *csum, *ctr;
    Segs seg;
};

size_t layout_group(void* ws, const GroupPlan& p, uint64_t m, size_t key_size, GroupWs* out) {
    Carver c(ws);
    GroupWs w{};
    const uint32_t D = 1u << p.bits;
    w.gq = c.take<char>(m * key_size);
    w.gpos = c.take<uint32_t>(m);
    w.gc = c.take<uint32_t>(m);
    w.mat = c.take<uint32_t>((size_t)p.ntiles * D);
    w.csum = c.take<uint32_t>((size_t)p.nchunks * D);
    w.ctr = c.take<uint32_t>(5);
    w.seg.seg_start = c.take<uint32_t>(2);
    w.seg.tile_prefix = c.take<uint32_t>(2);
    w.seg.chunk_prefix = c.take<uint32_t>(2);
    w.seg.S = 1;
    w.seg.ch = p.ch;
    if (out) *out = w;
    return c.off + 256;
}

}  // namespace

size_t probe_grouped_ws_bytes(uint64_t m, uint64_t V, size_t key_size) {
    return layout_group(nullptr, group_plan(m, V), m, key_size, nullptr);
}

template <typename Key>
hipError_t run_probe_grouped(const TableDev& t, const Key* queries, uint64_t m, uint32_t* counts,
                             unsigned long long* d_total, void* ws, hipStream_t s, bool decide) {
    if (m == 0) return run_probe_counts<Key>(t, queries, m, counts, d_total, s);
    HG_TRY(set_smem_limits<Key>());
    const GroupPlan p = group_plan(m, t.V);
    GroupWs w;
    layout_group(ws, p, m, sizeof(Key), &w);
    const auto hp = KeyTraits<Key>::make(t.V, t.seed);
    const uint32_t* gate = decide ? w.ctr : nullptr;  // ctr[0]: 1 grouped, 0 input order
    if (decide)
        hipLaunchKernelGGL(k_group_sample<Key>, dim3(1), dim3(1024), 0, s, queries, m, hp,
                           p.shift, p.bits, w.seg, p.ntiles, p.nchunks, w.ctr);
    else
        hipLaunchKernelGGL(k_segs_single, dim3(1), dim3(64), 0, s, w.seg, (uint32_t)m, p.ntiles,
                           p.nchunks, w.ctr);
    HG_TRY(hipGetLastError());
    Key* gq = (Key*)w.gq;
    // positions only when the counts go back to input order
    HG_TRY(partition_pass<Key>(queries, nullptr, gq, counts ? w.gpos : nullptr, w.seg, hp,
                               p.shift, p.bits, w.mat, w.csum, p.ntiles, p.nchunks, 3, false, s));
    // one probe launch: the grouped queries, or (gate 0) the queries in input
    // order straight into counts
    HG_TRY(run_probe_counts<Key>(t, gq, m, counts ? w.gc : nullptr, d_total, s, nullptr, true,
                                 gate, queries, counts));
    if (!counts) return hipSuccess;
    {
        HG_PROF("probe_ungroup", s);
        const uint32_t groups = (uint32_t)ceil_div(p.ntiles, kUngroupTiles);
        const uint32_t grid = (uint32_t)(8 * ceil_div(groups, 8));
        hipLaunchKernelGGL(k_ungroup_by_pos, dim3(grid), dim3(kUngroupThreads),
                           ungroup_smem(p.bits), s, m, p.ntiles, p.bits, (const uint32_t*)w.mat,
                           groups, (const uint32_t*)w.gpos, (const uint32_t*)w.gc, counts, gate);
    }
    return hipGetLastError();
}

template hipError_t run_probe_grouped<uint32_t>(const TableDev&, const uint32_t*, uint64_t,
                                                uint32_t*, unsigned long long*, void*,
                                                hipStream_t, bool);
template hipError_t run_probe_grouped<uint64_t>(const TableDev&, const uint64_t*, uint64_t,
                                                uint32_t*, unsigned long long*, void*,
                                                hipStream_t, bool);

template hipError_t run_build_v2<uint32_t>(const uint32_t*, uint64_t, uint64_t, uint64_t,
                                           uint32_t*, uint32_t*, uint32_t*, IndexOut&, void*,
                                           uint32_t, bool, hipStream_t);
template hipError_t run_build_v2<uint64_t>(const uint64_t*, uint64_t, uint64_t, uint64_t,
                                           uint32_t*, uint32_t*, uint64_t*, IndexOut&, void*,
                                           uint32_t, bool, hipStream_t);

}  // namespace hg
