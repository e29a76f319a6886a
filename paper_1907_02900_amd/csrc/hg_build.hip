// HashGraph builds on gfx950: Eq. 1 hashing, Alg. 1 (V1) and Alg. 2 (V2).
//
// V1 (Alg. 1) is written as the paper states it: a global atomic histogram,
// a prefix sum, and an atomic scatter that takes each key's slot from a cursor
// array initialised to the offsets.  On MI355X every device-scope atomic is
// executed beyond the L2, so V1 is bound by atomic throughput.
//
// V2 (Alg. 2) keeps the paper's idea -- first move keys into bins of
// contiguous bucket ranges so that the final placement is cache-local -- and
// maps it onto CDNA4 without global atomics:
//   * a final bin is a power-of-two range of 2^k buckets holding about 2048
//     keys on average, so that its keys, ids and bucket counters fit in LDS;
//   * keys reach their final bin by one or two stable partition passes over a
//     digit (a bit-field) of the bucket index.  Each pass is: per-tile digit
//     histograms (LDS), a segmented column scan of the tile x digit matrix
//     (giving every tile an exact base per digit, so no atomics and a
//     deterministic order), and a partition kernel that ranks a tile's keys by
//     digit with wave64 ballot matching and writes digit-contiguous runs;
//   * one workgroup per final bin then counts, scans and stably places the
//     bin's keys in LDS (two 6-bit ranking passes) and writes the bin's E
//     segment and offsets with coalesced stores.
// Every pass preserves input order among equal digits, so V2 places ids in
// ascending order inside each bucket: the result equals the stable layout.
#include "hg_internal.h"

namespace hg {

// ============================================================== hashing ===

template <typename Key>
__global__ void k_hash(const Key* __restrict__ keys, uint64_t n,
                       typename KeyTraits<Key>::Params hp, uint32_t* __restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) out[i] = KeyTraits<Key>::bucket(keys[i], hp);
}

static uint32_t stream_grid(uint64_t n, uint32_t block) {
    uint64_t g = ceil_div(n, (uint64_t)block * 4);
    if (g > 4096) g = 4096;
    if (g == 0) g = 1;
    return (uint32_t)g;
}

template <typename Key>
hipError_t run_hash(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* out,
                    hipStream_t s) {
    if (n == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(V, seed);
    {
        HG_PROF("hash", s);
        hipLaunchKernelGGL(k_hash<Key>, dim3(stream_grid(n, 256)), dim3(256), 0, s, keys, n, hp, out);
    }
    return hipGetLastError();
}

// ================================================================== V1 ===

template <typename Key>
__global__ void k_hist_global(const Key* __restrict__ keys, uint64_t n,
                              typename KeyTraits<Key>::Params hp, uint32_t* __restrict__ counts) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) atomic_add_relaxed(&counts[KeyTraits<Key>::bucket(keys[i], hp)], 1u);
}

template <typename Key>
__global__ void k_scatter_v1(const Key* __restrict__ keys, uint64_t n,
                             typename KeyTraits<Key>::Params hp, uint32_t* __restrict__ cursor,
                             uint32_t* __restrict__ ids, Key* __restrict__ ekeys) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        const Key k = keys[i];
        const uint32_t pos = atomic_add_relaxed_ret(&cursor[KeyTraits<Key>::bucket(k, hp)], 1u);
        if (pos < n) {  // always true when the counts are exact
            ekeys[pos] = k;
            ids[pos] = (uint32_t)i;
        }
    }
}

template <typename Key>
hipError_t run_histogram(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* counts,
                         uint32_t block, hipStream_t s) {
    if (!block) block = 256;
    HG_TRY(fill_u32(counts, V, 0u, s));
    if (n == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(V, seed);
    {
        HG_PROF("v1_hist_global", s);
        hipLaunchKernelGGL(k_hist_global<Key>, dim3(stream_grid(n, block)), dim3(block), 0, s, keys, n,
                           hp, counts);
    }
    return hipGetLastError();
}

template <typename Key>
hipError_t run_build_v1(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* offsets,
                        uint32_t* ids, Key* ekeys, void* ws, uint32_t block, hipStream_t s) {
    if (!block) block = 256;
    Carver c(ws);
    uint32_t* counts = c.take<uint32_t>(V);
    void* scan_ws = c.take<char>(scan_ws_bytes(V));
    HG_TRY(run_histogram<Key>(keys, n, V, seed, counts, block, s));
    // offsets = exclusive scan; the counts become the cursors (Alg. 1, fifth
    // loop re-zeroes them; here they start at the offsets so the scatter's
    // atomic returns the absolute slot).
    HG_TRY(scan_excl<uint32_t>(counts, V, offsets, counts, scan_ws, s));
    if (n == 0) return hipSuccess;
    auto hp = KeyTraits<Key>::make(V, seed);
    {
        HG_PROF("v1_scatter", s);
        hipLaunchKernelGGL(k_scatter_v1<Key>, dim3(stream_grid(n, block)), dim3(block), 0, s, keys, n,
                           hp, counts, ids, ekeys);
    }
    return hipGetLastError();
}

// ================================================================== V2 ===

// Segments of the source array, each cut into tiles of kPartTile entries, and
// the tiles grouped into chunks of `ch` consecutive tiles for the column scan.
struct Segs {
    uint32_t* seg_start;     // [S+1]
    uint32_t* tile_prefix;   // [S+1]
    uint32_t* chunk_prefix;  // [S+1]
    uint32_t S;
    uint32_t ch;
};

// largest s in [0, S) with pre[s] <= x (pre is non-decreasing, pre[0] = 0)
__device__ __forceinline__ uint32_t find_seg(const uint32_t* __restrict__ pre, uint32_t S, uint32_t x) {
    uint32_t lo = 0, hi = S;  // invariant: pre[lo] <= x, answer in [lo, hi)
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Tile `t` -> [begin, end) of the source; false if t is past the last tile.
__device__ __forceinline__ bool locate_tile(const Segs& g, uint32_t t, uint32_t& seg,
                                            uint32_t& begin, uint32_t& end) {
    if (t >= g.tile_prefix[g.S]) return false;
    seg = find_seg(g.tile_prefix, g.S, t);
    begin = g.seg_start[seg] + (t - g.tile_prefix[seg]) * kPartTile;
    const uint32_t se = g.seg_start[seg + 1];
    end = (se - begin > kPartTile) ? begin + kPartTile : se;
    return true;
}

// Blocks are dispatched round-robin over the 8 XCDs; map block b to a tile so
// that each XCD walks a contiguous range of tiles (adjacent tiles write
// adjacent parts of each digit's output range, which then merge in that XCD's
// L2).  Callers launch 8 * ceil(ub / 8) blocks.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t ub) {
    const uint32_t per = (ub + 7) >> 3;
    return (b & 7u) * per + (b >> 3);
}

template <typename Key>
__global__ __launch_bounds__(kPartThreads) void k_tile_hist(const Key* __restrict__ keys, Segs g,
                                                            typename KeyTraits<Key>::Params hp,
                                                            uint32_t shift, uint32_t bits,
                                                            uint32_t* __restrict__ mat,
                                                            uint32_t tiles_ub) {
    extern __shared__ uint32_t cnt[];
    const uint32_t D = 1u << bits;
    const uint32_t t = xcd_tile(blockIdx.x, tiles_ub);
    uint32_t seg, begin, end;
    if (!locate_tile(g, t, seg, begin, end)) return;
    for (uint32_t d = threadIdx.x; d < D; d += kPartThreads) cnt[d] = 0;
    __syncthreads();
    const uint32_t mask = D - 1;
    for (uint32_t i = begin + threadIdx.x; i < end; i += kPartThreads) {
        const uint32_t d = (KeyTraits<Key>::bucket(keys[i], hp) >> shift) & mask;
        atomicAdd(&cnt[d], 1u);
    }
    __syncthreads();
    uint32_t* row = mat + (size_t)t * D;
    for (uint32_t d = threadIdx.x; d < D; d += kPartThreads) row[d] = cnt[d];
}

// ---- segmented column scan of the [tile][digit] matrix ----------------------
// base(t, d) = seg_start[s] + sum_{d' < d} total_s(d') + sum_{t' < t in s} M[t'][d]
// i.e. the exclusive prefix in (segment, digit, tile) order, which is where
// tile t's keys of digit d go in the stably partitioned output.

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
        for (uint32_t t = t0; t < t1; ++t) s += mat[(size_t)t * D + d];
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
    // each thread owns D/256 consecutive digits (D >= 256) or one digit
    const uint32_t per = (D + 255) / 256;
    const uint32_t d0 = threadIdx.x * per;
    uint32_t tot[8];  // D <= 2048
    uint32_t mine = 0;
    for (uint32_t j = 0; j < per; ++j) {
        uint32_t d = d0 + j, acc = 0;
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
                uint32_t v = csum[(size_t)c * D + d];
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
        for (uint32_t t = t0; t < t1; ++t) {
            uint32_t v = mat[(size_t)t * D + d];
            mat[(size_t)t * D + d] = r;
            r += v;
        }
    }
}

// ---- stable ranking of a tile by a digit -------------------------------------
// Items are wave-striped: wave w owns entries [w*64*ITEMS, (w+1)*64*ITEMS) and
// takes them 64 at a time, so processing order equals entry order.  For each
// round, lanes with equal digits are found with `bits` ballots; the lowest
// such lane bumps the wave's counter for that digit.  After all rounds the
// (digit, wave) counters are scanned digit-major, giving each item its
// position in the stably sorted tile.  Invalid items carry digit >= D.
template <int THREADS, int ITEMS>
__device__ __forceinline__ void rank_by_digit(const uint32_t (&dig)[ITEMS], uint32_t bits,
                                              uint32_t* wcnt /* W*D */, uint32_t* dstart /* D */,
                                              uint32_t* tmp, uint32_t (&pos)[ITEMS]) {
    constexpr int W = THREADS / kWave;
    const uint32_t D = 1u << bits;
    const uint32_t w = threadIdx.x / kWave;
    for (uint32_t i = threadIdx.x; i < W * D; i += THREADS) wcnt[i] = 0;
    __syncthreads();
    uint32_t* my = wcnt + w * D;
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const bool valid = dig[r] < D;
        const uint64_t vm = ballot(valid);
        if (vm == 0) continue;
        const uint64_t peers = match_digit(dig[r], (int)bits, vm);
        if (valid) {
            const uint32_t below = mbcnt(peers);
            const uint32_t old = my[dig[r]];
            if (below == 0) my[dig[r]] = old + (uint32_t)__popcll(peers);
            pos[r] = old + below;
        }
    }
    __syncthreads();
    // digit-major scan of the (digit, wave) counters
    const uint32_t per = (D + THREADS - 1) / THREADS;
    const uint32_t d0 = threadIdx.x * per;
    uint32_t mine = 0;
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t d = d0 + j;
        if (d < D)
            for (int ww = 0; ww < W; ++ww) mine += wcnt[ww * D + d];
    }
    uint32_t all;
    uint32_t run = block_excl_scan<THREADS>(mine, tmp, &all);
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t d = d0 + j;
        if (d < D) {
            dstart[d] = run;
            for (int ww = 0; ww < W; ++ww) {
                const uint32_t v = wcnt[ww * D + d];
                wcnt[ww * D + d] = run;
                run += v;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
        if (dig[r] < D) pos[r] += my[dig[r]];
}

// Stable partition of one tile by a digit of the bucket index.  Writes every
// entry to base(tile, digit) + its rank among the tile's entries of that digit.
template <typename Key, bool HAS_IDS>
__global__ __launch_bounds__(kPartThreads) void k_tile_partition(
    const Key* __restrict__ src_keys, const uint32_t* __restrict__ src_ids,
    Key* __restrict__ dst_keys, uint32_t* __restrict__ dst_ids, Segs g,
    typename KeyTraits<Key>::Params hp, uint32_t shift, uint32_t bits,
    const uint32_t* __restrict__ base, uint32_t tiles_ub) {
    constexpr int W = kPartThreads / kWave;
    constexpr int IT = kPartItems;
    const uint32_t D = 1u << bits;
    extern __shared__ __align__(16) unsigned char smem[];
    Key* skeys = (Key*)smem;
    uint32_t* sids = (uint32_t*)(skeys + kPartTile);
    uint16_t* sdig = (uint16_t*)(sids + kPartTile);
    uint32_t* wcnt = (uint32_t*)(sdig + kPartTile);
    uint32_t* dstart = wcnt + W * D;
    uint32_t* tbase = dstart + D;
    uint32_t* tmp = tbase + D;

    const uint32_t t = xcd_tile(blockIdx.x, tiles_ub);
    uint32_t seg, begin, end;
    if (!locate_tile(g, t, seg, begin, end)) return;
    const uint32_t cnt = end - begin;
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t mask = D - 1;

    Key k[IT];
    uint32_t id[IT], dig[IT], pos[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t e = w * (kWave * IT) + r * kWave + lane;
        if (e < cnt) {
            k[r] = src_keys[begin + e];
            id[r] = HAS_IDS ? src_ids[begin + e] : begin + e;
        } else {
            k[r] = 0;
            id[r] = 0;
        }
    }
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint32_t e = w * (kWave * IT) + r * kWave + lane;
        dig[r] = (e < cnt) ? ((KeyTraits<Key>::bucket(k[r], hp) >> shift) & mask) : D;
    }
    rank_by_digit<kPartThreads, IT>(dig, bits, wcnt, dstart, tmp, pos);
    const uint32_t* row = base + (size_t)t * D;
    for (uint32_t d = threadIdx.x; d < D; d += kPartThreads) tbase[d] = row[d] - dstart[d];
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
            dst_ids[o] = sids[p];
        }
    }
}

template <typename Key>
static size_t partition_smem(uint32_t bits) {
    const size_t D = 1u << bits;
    return kPartTile * (sizeof(Key) + 4 + 2) + (kPartThreads / kWave) * D * 4 + 2 * D * 4 +
           (kPartThreads / kWave + 1) * 4 + 64;
}

// Tier-1 segment: the whole input.
__global__ void k_segs_single(Segs g, uint32_t n, uint32_t ntiles, uint32_t nchunks) {
    if (threadIdx.x == 0) {
        g.seg_start[0] = 0;
        g.seg_start[1] = n;
        g.tile_prefix[0] = 0;
        g.tile_prefix[1] = ntiles;
        g.chunk_prefix[0] = 0;
        g.chunk_prefix[1] = nchunks;
    }
}

// Tier-2 segments: one per tier-1 digit, taken from row 0 of the scanned
// tier-1 matrix (the start of every digit's range).  One workgroup of 1024
// threads; S <= 2048.
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

// Start of every final bin (bin = segment * D + digit) in the partitioned
// array, plus bin_start[bins] = n.
__global__ void k_bin_starts(const uint32_t* __restrict__ base, Segs g, uint32_t bits,
                             uint32_t bins, uint32_t n, uint32_t* __restrict__ bin_start) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > bins) return;
    if (b == bins) {
        bin_start[b] = n;
        return;
    }
    const uint32_t D = 1u << bits;
    const uint32_t s = b >> bits, d = b & (D - 1);
    const uint32_t t0 = g.tile_prefix[s];
    bin_start[b] = (g.tile_prefix[s + 1] > t0) ? base[(size_t)t0 * D + d] : g.seg_start[s];
}

// ---- per-bin LDS build (Alg. 2 phase 3) -------------------------------------
// One workgroup per final bin g, covering buckets [g*2^k, min((g+1)*2^k, V)).
// The bin's entries are loaded (in order), counted per bucket, stably sorted by
// local bucket with two LSD ranking passes, and written back as the bin's E
// segment; the bucket counts are scanned into the bin's offsets.  A bin larger
// than the LDS capacity (only under heavy skew) is processed in capacity-sized
// chunks with running per-bucket cursors, still in order.
template <typename Key>
__global__ __launch_bounds__(kLocalThreads) void k_local_build(
    const Key* __restrict__ src_keys, const uint32_t* __restrict__ src_ids,
    const uint32_t* __restrict__ bin_start, typename KeyTraits<Key>::Params hp, uint32_t k,
    uint32_t n, uint32_t* __restrict__ offsets, uint32_t* __restrict__ ids,
    Key* __restrict__ ekeys) {
    constexpr int W = kLocalThreads / kWave;
    constexpr int IT = kLocalItems;
    constexpr uint32_t CAP = kLocalCap;
    const uint32_t NB = 1u << k;                     // buckets per bin
    const uint32_t lo_bits = (k + 1) / 2, hi_bits = k / 2;
    const uint32_t DR = 1u << (lo_bits > hi_bits ? lo_bits : hi_bits);
    extern __shared__ __align__(16) unsigned char smem[];
    Key* skeys = (Key*)smem;
    uint32_t* sids = (uint32_t*)(skeys + CAP);
    uint16_t* sb = (uint16_t*)(sids + CAP);
    uint32_t* cnt = (uint32_t*)(sb + CAP);   // NB: per-bucket counts / cursors
    uint32_t* tcnt = cnt + NB;               // NB: per-chunk counts (heavy path)
    uint32_t* wcnt = tcnt + NB;              // W * DR
    uint32_t* dstart = wcnt + W * DR;        // DR
    uint32_t* tmp = dstart + DR;

    const uint32_t g = blockIdx.x;
    const uint32_t start = bin_start[g], end = bin_start[g + 1];
    const uint32_t L = end - start;
    const uint32_t v0 = g << k;
    const uint32_t V = hp.range;
    const uint32_t nb = (V - v0 < NB) ? V - v0 : NB;
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();

    for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads) cnt[i] = 0;
    __syncthreads();
    const bool heavy = L > CAP;
    if (heavy) {
        for (uint32_t i = start + threadIdx.x; i < end; i += kLocalThreads)
            atomicAdd(&cnt[KeyTraits<Key>::bucket(src_keys[i], hp) - v0], 1u);
        __syncthreads();
    }

    // process the bin in chunks of CAP entries (exactly one chunk when light)
    const uint32_t nchunk = L ? (uint32_t)(((uint64_t)L + CAP - 1) / CAP) : 1u;
    for (uint32_t ci = 0; ci < nchunk; ++ci) {
        const uint32_t c0 = ci * CAP;
        const uint32_t cl = (L - c0 < CAP) ? L - c0 : CAP;
        Key kk[IT];
        uint32_t id[IT], b[IT], pos[IT], dig[IT];
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const uint32_t e = w * (kWave * IT) + r * kWave + lane;
            if (e < cl) {
                kk[r] = src_keys[start + c0 + e];
                id[r] = src_ids[start + c0 + e];
            } else {
                kk[r] = 0;
                id[r] = 0;
            }
        }
        if (heavy) {
            for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads) tcnt[i] = 0;
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const uint32_t e = w * (kWave * IT) + r * kWave + lane;
            if (e < cl) {
                b[r] = KeyTraits<Key>::bucket(kk[r], hp) - v0;
                atomicAdd(heavy ? &tcnt[b[r]] : &cnt[b[r]], 1u);
            } else {
                b[r] = NB;
            }
        }
        if (k > 0) {
            // pass 1: low bits
#pragma unroll
            for (int r = 0; r < IT; ++r) dig[r] = (b[r] < NB) ? (b[r] & ((1u << lo_bits) - 1)) : DR;
            rank_by_digit<kLocalThreads, IT>(dig, lo_bits, wcnt, dstart, tmp, pos);
#pragma unroll
            for (int r = 0; r < IT; ++r)
                if (b[r] < NB) {
                    skeys[pos[r]] = kk[r];
                    sids[pos[r]] = id[r];
                    sb[pos[r]] = (uint16_t)b[r];
                }
            __syncthreads();
            if (hi_bits > 0) {
#pragma unroll
                for (int r = 0; r < IT; ++r) {
                    const uint32_t e = w * (kWave * IT) + r * kWave + lane;
                    if (e < cl) {
                        kk[r] = skeys[e];
                        id[r] = sids[e];
                        b[r] = sb[e];
                        dig[r] = b[r] >> lo_bits;
                    } else {
                        dig[r] = DR;
                    }
                }
                // rank_by_digit starts with a barrier, so the reads above are
                // complete before the buffers are overwritten below
                rank_by_digit<kLocalThreads, IT>(dig, hi_bits, wcnt, dstart, tmp, pos);
#pragma unroll
                for (int r = 0; r < IT; ++r)
                    if (dig[r] < DR) {
                        skeys[pos[r]] = kk[r];
                        sids[pos[r]] = id[r];
                        sb[pos[r]] = (uint16_t)b[r];
                    }
            }
        } else {
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                const uint32_t e = w * (kWave * IT) + r * kWave + lane;
                if (e < cl) {
                    skeys[e] = kk[r];
                    sids[e] = id[r];
                    sb[e] = 0;
                }
            }
        }
        __syncthreads();

        if (!heavy) {
            // offsets of this bin's buckets and the E segment, coalesced
            const uint32_t per = NB / kLocalThreads ? NB / kLocalThreads : 1u;
            const uint32_t i0 = threadIdx.x * per;
            uint32_t mine = 0;
            for (uint32_t j = 0; j < per; ++j)
                if (i0 + j < NB) mine += cnt[i0 + j];
            uint32_t all;
            uint32_t run = start + block_excl_scan<kLocalThreads>(mine, tmp, &all);
            for (uint32_t j = 0; j < per; ++j)
                if (i0 + j < nb) {
                    offsets[v0 + i0 + j] = run;
                    run += cnt[i0 + j];
                }
            for (uint32_t p = threadIdx.x; p < cl; p += kLocalThreads) {
                ekeys[start + p] = skeys[p];
                ids[start + p] = sids[p];
            }
        } else {
            if (c0 == 0) {
                // bucket bases of the whole bin -> offsets and cursors
                const uint32_t per = NB / kLocalThreads ? NB / kLocalThreads : 1u;
                const uint32_t i0 = threadIdx.x * per;
                uint32_t mine = 0;
                for (uint32_t j = 0; j < per; ++j)
                    if (i0 + j < NB) mine += cnt[i0 + j];
                uint32_t all;
                uint32_t run = start + block_excl_scan<kLocalThreads>(mine, tmp, &all);
                for (uint32_t j = 0; j < per; ++j)
                    if (i0 + j < NB) {
                        const uint32_t v = cnt[i0 + j];
                        cnt[i0 + j] = run;
                        if (i0 + j < nb) offsets[v0 + i0 + j] = run;
                        run += v;
                    }
            }
            // chunk-local bucket starts (exclusive scan of tcnt) -> tcnt
            {
                const uint32_t per = NB / kLocalThreads ? NB / kLocalThreads : 1u;
                const uint32_t i0 = threadIdx.x * per;
                uint32_t mine = 0;
                for (uint32_t j = 0; j < per; ++j)
                    if (i0 + j < NB) mine += tcnt[i0 + j];
                uint32_t all;
                uint32_t run = block_excl_scan<kLocalThreads>(mine, tmp, &all);
                __syncthreads();
                for (uint32_t j = 0; j < per; ++j)
                    if (i0 + j < NB) {
                        const uint32_t v = tcnt[i0 + j];
                        tcnt[i0 + j] = run;
                        run += v;
                    }
            }
            __syncthreads();
            for (uint32_t p = threadIdx.x; p < cl; p += kLocalThreads) {
                const uint32_t bb = sb[p];
                const uint32_t o = cnt[bb] + (p - tcnt[bb]);
                if (o - start < L) {
                    ekeys[o] = skeys[p];
                    ids[o] = sids[p];
                }
            }
            __syncthreads();
            // advance the cursors by this chunk's counts: the count of bucket
            // bb in the chunk is (next start - start), recomputed from tcnt
            for (uint32_t i = threadIdx.x; i < NB; i += kLocalThreads) {
                const uint32_t nxt = (i + 1 < NB) ? tcnt[i + 1] : cl;
                cnt[i] += nxt - tcnt[i];
            }
            __syncthreads();
        }
    }
    if (g == gridDim.x - 1 && threadIdx.x == 0) offsets[V] = n;
}

template <typename Key>
static size_t local_smem(uint32_t k) {
    const size_t NB = 1u << k;
    const uint32_t lo = (k + 1) / 2;
    const size_t DR = 1u << lo;
    return kLocalCap * (sizeof(Key) + 4 + 2) + 2 * NB * 4 + (kLocalThreads / kWave) * DR * 4 +
           DR * 4 + (kLocalThreads / kWave + 1) * 4 + 64;
}

// ---- plan --------------------------------------------------------------------

V2Plan plan_v2(uint64_t n, uint64_t V, int key_bits, uint32_t bins_hint) {
    (void)key_bits;
    V2Plan p;
    p.n = n;
    p.V = V;
    uint32_t k;
    if (bins_hint) {
        k = log2_ceil(ceil_div(V, bins_hint));
    } else if (n == 0) {
        k = kMaxLocalBits;
    } else {
        // about 2048 keys per final bin: 2^k * n / V ~ 2048
        const double r = 2048.0 * (double)V / (double)n;
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
        p.b1 = (bits + 1) / 2;
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

struct V2Ws {
    void* rkeys;
    uint32_t* rids;
    uint32_t *m1, *c1, *m2, *c2, *bin_start;
    Segs s1, s2;
};

static V2Ws carve_v2(void* ws, const V2Plan& p, size_t key_size) {
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
    w.rids = w.rids;
    (void)c.take<char>(0);
    return w;
}

size_t build_ws_bytes(int variant, uint64_t n, uint64_t V, int key_bits, uint32_t bins_hint) {
    const size_t ks = key_bits == 64 ? 8 : 4;
    if (variant == 1) {
        Carver c(nullptr);
        c.take<uint32_t>(V);
        c.take<char>(scan_ws_bytes(V));
        return c.off + 256;
    }
    V2Plan p = plan_v2(n, V, key_bits, bins_hint);
    Carver c(nullptr);
    c.take<char>(n * ks);
    c.take<uint32_t>(n);
    const uint32_t D1 = 1u << p.b1, D2 = 1u << p.b2;
    c.take<uint32_t>((size_t)p.ntiles1 * D1);
    c.take<uint32_t>((size_t)p.nchunks1 * D1);
    c.take<uint32_t>(2);
    c.take<uint32_t>(2);
    c.take<uint32_t>(2);
    if (p.tiers == 2) {
        c.take<uint32_t>((size_t)p.ntiles2_ub * D2);
        c.take<uint32_t>((size_t)p.nchunks2_ub * D2);
        c.take<uint32_t>(D1 + 1);
        c.take<uint32_t>(D1 + 1);
        c.take<uint32_t>(D1 + 1);
    }
    c.take<uint32_t>((size_t)p.bins + 1);
    return c.off + 256;
}

static hipError_t colscan(uint32_t* mat, const Segs& g, uint32_t D, uint32_t* csum,
                          uint32_t nchunks_ub, hipStream_t s) {
    {
        HG_PROF("v2_colscan_reduce", s);
        hipLaunchKernelGGL(k_colscan_reduce, dim3(nchunks_ub), dim3(256), 0, s, (const uint32_t*)mat, g,
                           D, csum);
    }
    HG_TRY(hipGetLastError());
    {
        HG_PROF("v2_colscan_seg", s);
        hipLaunchKernelGGL(k_colscan_seg, dim3(g.S), dim3(256), 0, s, g, D, csum);
    }
    HG_TRY(hipGetLastError());
    {
        HG_PROF("v2_colscan_down", s);
        hipLaunchKernelGGL(k_colscan_down, dim3(nchunks_ub), dim3(256), 0, s, mat, g, D,
                           (const uint32_t*)csum);
    }
    return hipGetLastError();
}

template <typename Key>
static hipError_t partition_pass(const Key* src_keys, const uint32_t* src_ids, Key* dst_keys,
                                 uint32_t* dst_ids, const Segs& g,
                                 typename KeyTraits<Key>::Params hp, uint32_t shift,
                                 uint32_t bits, uint32_t* mat, uint32_t* csum, uint32_t tiles_ub,
                                 uint32_t nchunks_ub, int tier, hipStream_t s) {
    const uint32_t D = 1u << bits;
    const uint32_t grid = (uint32_t)(8 * ceil_div(tiles_ub, 8));
    {
        HG_PROF(tier == 1 ? "v2_tile_hist_t1" : "v2_tile_hist_t2", s);
        hipLaunchKernelGGL(k_tile_hist<Key>, dim3(grid), dim3(kPartThreads), D * 4, s, src_keys, g, hp,
                           shift, bits, mat, tiles_ub);
    }
    HG_TRY(hipGetLastError());
    HG_TRY(colscan(mat, g, D, csum, nchunks_ub, s));
    const size_t smem = partition_smem<Key>(bits);
    if (src_ids) {
        {
            HG_PROF(tier == 1 ? "v2_partition_t1" : "v2_partition_t2", s);
            hipLaunchKernelGGL((k_tile_partition<Key, true>), dim3(grid), dim3(kPartThreads), smem, s,
                               src_keys, src_ids, dst_keys, dst_ids, g, hp, shift, bits,
                               (const uint32_t*)mat, tiles_ub);
        }
    } else {
        {
            HG_PROF(tier == 1 ? "v2_partition_t1" : "v2_partition_t2", s);
            hipLaunchKernelGGL((k_tile_partition<Key, false>), dim3(grid), dim3(kPartThreads), smem, s,
                               src_keys, src_ids, dst_keys, dst_ids, g, hp, shift, bits,
                               (const uint32_t*)mat, tiles_ub);
        }
    }
    return hipGetLastError();
}

template <typename Key>
static hipError_t set_smem_limits() {
    static bool done = false;
    if (done) return hipSuccess;
    HG_TRY(hipFuncSetAttribute((const void*)k_tile_partition<Key, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    HG_TRY(hipFuncSetAttribute((const void*)k_tile_partition<Key, false>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    HG_TRY(hipFuncSetAttribute((const void*)k_local_build<Key>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    done = true;
    return hipSuccess;
}

template <typename Key>
hipError_t run_build_v2(const Key* keys, uint64_t n, uint64_t V, uint64_t seed, uint32_t* offsets,
                        uint32_t* ids, Key* ekeys, void* ws, uint32_t bins_hint, hipStream_t s) {
    HG_TRY(set_smem_limits<Key>());
    if (n == 0) return fill_u32(offsets, V + 1, 0u, s);
    const V2Plan p = plan_v2(n, V, sizeof(Key) * 8, bins_hint);
    V2Ws w = carve_v2(ws, p, sizeof(Key));
    auto hp = KeyTraits<Key>::make(V, seed);
    Key* rkeys = (Key*)w.rkeys;

    {
        HG_PROF("v2_segs", s);
        hipLaunchKernelGGL(k_segs_single, dim3(1), dim3(64), 0, s, w.s1, (uint32_t)n, p.ntiles1,
                           p.nchunks1);
    }
    HG_TRY(hipGetLastError());
    const Key* bin_keys;
    const uint32_t* bin_ids;
    if (p.tiers == 1) {
        HG_TRY(partition_pass<Key>(keys, nullptr, rkeys, w.rids, w.s1, hp, p.k, p.b1, w.m1, w.c1,
                                   p.ntiles1, p.nchunks1, 1, s));
        {
            HG_PROF("v2_bin_starts", s);
            hipLaunchKernelGGL(k_bin_starts, dim3((uint32_t)ceil_div(p.bins + 1, 256)), dim3(256), 0, s,
                               (const uint32_t*)w.m1, w.s1, p.b1, p.bins, (uint32_t)n, w.bin_start);
        }
        HG_TRY(hipGetLastError());
        bin_keys = rkeys;
        bin_ids = w.rids;
    } else {
        // tier 1 into the table's own arrays, tier 2 into the workspace
        HG_TRY(partition_pass<Key>(keys, nullptr, ekeys, ids, w.s1, hp, p.k + p.b2, p.b1, w.m1,
                                   w.c1, p.ntiles1, p.nchunks1, 1, s));
        {
            HG_PROF("v2_segs", s);
            hipLaunchKernelGGL(k_segs_from_bases, dim3(1), dim3(1024), 0, s, (const uint32_t*)w.m1,
                               p.ntiles1, (uint32_t)n, w.s2);
        }
        HG_TRY(hipGetLastError());
        HG_TRY(partition_pass<Key>(ekeys, ids, rkeys, w.rids, w.s2, hp, p.k, p.b2, w.m2, w.c2,
                                   p.ntiles2_ub, p.nchunks2_ub, 2, s));
        {
            HG_PROF("v2_bin_starts", s);
            hipLaunchKernelGGL(k_bin_starts, dim3((uint32_t)ceil_div(p.bins + 1, 256)), dim3(256), 0, s,
                               (const uint32_t*)w.m2, w.s2, p.b2, p.bins, (uint32_t)n, w.bin_start);
        }
        HG_TRY(hipGetLastError());
        bin_keys = rkeys;
        bin_ids = w.rids;
    }
    {
        HG_PROF("v2_local_build", s);
        hipLaunchKernelGGL(k_local_build<Key>, dim3(p.bins), dim3(kLocalThreads), local_smem<Key>(p.k),
                           s, bin_keys, bin_ids, (const uint32_t*)w.bin_start, hp, p.k, (uint32_t)n,
                           offsets, ids, ekeys);
    }
    return hipGetLastError();
}

#define HG_INST(Key)                                                                              \
    template hipError_t run_hash<Key>(const Key*, uint64_t, uint64_t, uint64_t, uint32_t*,       \
                                      hipStream_t);                                              \
    template hipError_t run_histogram<Key>(const Key*, uint64_t, uint64_t, uint64_t, uint32_t*,  \
                                           uint32_t, hipStream_t);                               \
    template hipError_t run_build_v1<Key>(const Key*, uint64_t, uint64_t, uint64_t, uint32_t*,   \
                                          uint32_t*, Key*, void*, uint32_t, hipStream_t);        \
    template hipError_t run_build_v2<Key>(const Key*, uint64_t, uint64_t, uint64_t, uint32_t*,   \
                                          uint32_t*, Key*, void*, uint32_t, hipStream_t);
HG_INST(uint32_t)
HG_INST(uint64_t)

}  // namespace hg
