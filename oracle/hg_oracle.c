/*
 * CPU oracle for the HashGraph hot path
 * (O. Green, "HashGraph -- Scalable Hash Tables Using A Sparse Graph Data
 * Structure", arXiv:1907.02900).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  This file is the plain, slow,
 * sequential definition that the GPU library is checked against.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it.  It shares no source with the HIP library: its hash finalisers, its
 * modulo (native '%') and its sort are written here and nowhere else.
 *
 * Everything is integer arithmetic; there is no rounding anywhere.
 *
 * What each entry point follows (sections, equations and algorithms of the
 * paper):
 *   orc_fmix32, orc_fmix64  the MurmurHash3 finalisers (Appleby), the hash
 *                           family the paper names for Eq. 1 (Sec. 2,
 *                           "Hashing").  32-bit keys use fmix32, 64-bit keys
 *                           fmix64; the seed is XOR-ed into the key first.
 *   orc_hash                Eq. 1: bucket = hash(key) mod V, range 0..V-1.
 *   orc_count               Alg. 1, second and third loops: zeroed counters,
 *                           one increment per key.
 *   orc_exclusive_scan      Alg. 1 PrefixSum, producing the CSR offset array
 *                           of Sec. 3.1 (V+1 entries, offsets[V] == N).
 *   orc_place               Alg. 1 last loop, read with the base offset that
 *                           Sec. 3.2 step 6 describes: position = offset of
 *                           the bucket + running rank inside it.  Keys are
 *                           visited in ascending input order, so ids end up
 *                           ascending inside each bucket: this is the stable
 *                           layout.
 *   orc_build               orc_hash + orc_count + orc_exclusive_scan +
 *                           orc_place, i.e. the table both Alg. 1 and Alg. 2
 *                           produce (Sec. 1 contributions, Sec. 5.1: both
 *                           variants give the same table up to the order
 *                           inside a bucket).
 *   orc_probe_counts        Sec. 3.4 HashGraph-Probe-Standard reports every
 *                           instance of a query key (Sec. 5.2), so the result
 *                           is count[j] = #{ i : key[i] == query[j] }.  It is
 *                           computed WITHOUT the hash, by sorting both sides
 *                           and merging, so that it does not depend on V,
 *                           seed or variant.
 *   orc_probe_pairs         the matching (build id, probe id) pairs in the
 *                           canonical order (probe id ascending, then build
 *                           id ascending).
 *   orc_count_one           brute-force count of one query by a full scan,
 *                           for sampled checks on very large inputs.
 *
 * Alg. 3 (HashGraph-Probe-New) intersects bucket x of table A with bucket x of
 * table B for every x.  Because both tables use the same hash and V, equal
 * keys always meet in the same bucket, so its result is the probe result with
 * B's keys as the queries; the tests use orc_probe_counts/orc_probe_pairs for
 * it.
 *
 * Pins (checks against something other than this file) live in
 * tests/test_oracle_pins.py.  fmix64's constants are pinned by published
 * MurmurHash3_x64_128 outputs and fmix32's by MurmurHash3_x86_32 outputs
 * (tests/golden/murmur3_vectors.txt).
 *
 * Return codes: 0 ok, 1 invalid argument, 2 out of memory, 3 capacity too
 * small (the total is still reported).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2
#define ORC_ECAPACITY 3

/* ---- Eq. 1: the hash ------------------------------------------------- */

uint32_t orc_fmix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

uint64_t orc_fmix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

/* bucket of one key: (fmix(key ^ seed)) mod V, computed with native '%'.
 * 32-bit keys use the low 32 bits of the seed. */
uint32_t orc_bucket_one(uint64_t key, int key_bits, uint64_t V, uint64_t seed)
{
    if (key_bits == 32) {
        uint32_t h = orc_fmix32((uint32_t)key ^ (uint32_t)seed);
        return (uint32_t)((uint64_t)h % V);
    }
    return (uint32_t)(orc_fmix64(key ^ seed) % V);
}

static int valid_args(int key_bits, uint64_t V)
{
    return (key_bits == 32 || key_bits == 64) && V >= 1 && V <= 0xffffffffull;
}

static uint64_t key_at(const void *keys, int key_bits, uint64_t i)
{
    return key_bits == 32 ? (uint64_t)((const uint32_t *)keys)[i]
                          : ((const uint64_t *)keys)[i];
}

static void key_put(void *keys, int key_bits, uint64_t i, uint64_t k)
{
    if (key_bits == 32)
        ((uint32_t *)keys)[i] = (uint32_t)k;
    else
        ((uint64_t *)keys)[i] = k;
}

int orc_hash(const void *keys, uint64_t n, int key_bits, uint64_t V, uint64_t seed,
             uint32_t *h)
{
    if (!valid_args(key_bits, V))
        return ORC_EINVAL;
    for (uint64_t i = 0; i < n; ++i)
        h[i] = orc_bucket_one(key_at(keys, key_bits, i), key_bits, V, seed);
    return ORC_OK;
}

/* ---- Alg. 1: count, prefix sum, place --------------------------------- */

int orc_count(const uint32_t *h, uint64_t n, uint64_t V, uint32_t *counts)
{
    for (uint64_t b = 0; b < V; ++b)
        counts[b] = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (h[i] >= V)
            return ORC_EINVAL;
        counts[h[i]] += 1;
    }
    return ORC_OK;
}

/* offsets[0] = 0, offsets[b+1] = offsets[b] + counts[b]; V+1 entries. */
int orc_exclusive_scan(const uint32_t *counts, uint64_t V, uint32_t *offsets)
{
    uint64_t run = 0;
    for (uint64_t b = 0; b < V; ++b) {
        offsets[b] = (uint32_t)run;
        run += counts[b];
    }
    offsets[V] = (uint32_t)run;
    return run > 0xffffffffull ? ORC_EINVAL : ORC_OK;
}

/* Visit keys in input order; each goes to offset-of-its-bucket plus the
 * number of earlier keys already placed in that bucket. */
int orc_place(const void *keys, const uint32_t *h, uint64_t n, int key_bits, uint64_t V,
              const uint32_t *offsets, uint32_t *ids, void *ekeys)
{
    uint32_t *cursor = (uint32_t *)malloc((V ? V : 1) * sizeof(uint32_t));
    if (!cursor)
        return ORC_ENOMEM;
    memcpy(cursor, offsets, V * sizeof(uint32_t));
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t p = cursor[h[i]]++;
        ids[p] = (uint32_t)i;
        key_put(ekeys, key_bits, p, key_at(keys, key_bits, i));
    }
    free(cursor);
    return ORC_OK;
}

int orc_build(const void *keys, uint64_t n, int key_bits, uint64_t V, uint64_t seed,
              uint32_t *offsets, uint32_t *ids, void *ekeys)
{
    if (!valid_args(key_bits, V) || n > 0xffffffffull)
        return ORC_EINVAL;
    uint32_t *h = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *counts = (uint32_t *)malloc(V * sizeof(uint32_t));
    int rc = ORC_ENOMEM;
    if (h && counts) {
        rc = orc_hash(keys, n, key_bits, V, seed, h);
        if (rc == ORC_OK)
            rc = orc_count(h, n, V, counts);
        if (rc == ORC_OK)
            rc = orc_exclusive_scan(counts, V, offsets);
        if (rc == ORC_OK)
            rc = orc_place(keys, h, n, key_bits, V, offsets, ids, ekeys);
    }
    free(h);
    free(counts);
    return rc;
}

/* ---- probing, defined by key equality (no hash) ------------------------ */

/* Stable LSD radix sort of (key, index) pairs by key, 8 bits per pass.  Keys
 * are widened to 64 bits; 32-bit keys take 4 passes, 64-bit keys 8.  Output:
 * sorted keys and the original indices (ascending among equal keys). */
static int sort_pairs(const void *keys, uint64_t n, int key_bits, uint64_t **out_k,
                      uint32_t **out_i)
{
    size_t nn = n ? n : 1;
    uint64_t *k0 = (uint64_t *)malloc(nn * sizeof(uint64_t));
    uint64_t *k1 = (uint64_t *)malloc(nn * sizeof(uint64_t));
    uint32_t *i0 = (uint32_t *)malloc(nn * sizeof(uint32_t));
    uint32_t *i1 = (uint32_t *)malloc(nn * sizeof(uint32_t));
    if (!k0 || !k1 || !i0 || !i1) {
        free(k0); free(k1); free(i0); free(i1);
        return ORC_ENOMEM;
    }
    for (uint64_t i = 0; i < n; ++i) {
        k0[i] = key_at(keys, key_bits, i);
        i0[i] = (uint32_t)i;
    }
    int passes = key_bits / 8;
    for (int pass = 0; pass < passes; ++pass) {
        int shift = 8 * pass;
        uint64_t cnt[257];
        memset(cnt, 0, sizeof(cnt));
        for (uint64_t i = 0; i < n; ++i)
            cnt[((k0[i] >> shift) & 0xff) + 1] += 1;
        for (int d = 0; d < 256; ++d)
            cnt[d + 1] += cnt[d];
        for (uint64_t i = 0; i < n; ++i) {
            uint64_t p = cnt[(k0[i] >> shift) & 0xff]++;
            k1[p] = k0[i];
            i1[p] = i0[i];
        }
        uint64_t *tk = k0; k0 = k1; k1 = tk;
        uint32_t *ti = i0; i0 = i1; i1 = ti;
    }
    free(k1);
    free(i1);
    *out_k = k0;
    *out_i = i0;
    return ORC_OK;
}

/* count[j] = #{i : key[i] == query[j]}; also, when run_start is not NULL,
 * run_start[j] = first index of key query[j] in the key-sorted order and
 * *sorted_ids_out = the build ids in key-sorted order (caller frees). */
static int probe_core(const void *keys, uint64_t n, const void *queries, uint64_t m,
                      int key_bits, uint32_t *counts, uint32_t *run_start,
                      uint32_t **sorted_ids_out, uint64_t *total)
{
    if (!(key_bits == 32 || key_bits == 64) || n > 0xffffffffull || m > 0xffffffffull)
        return ORC_EINVAL;
    uint64_t *sk = NULL, *sq = NULL;
    uint32_t *si = NULL, *sj = NULL;
    int rc = sort_pairs(keys, n, key_bits, &sk, &si);
    if (rc == ORC_OK)
        rc = sort_pairs(queries, m, key_bits, &sq, &sj);
    if (rc != ORC_OK) {
        free(sk); free(si); free(sq); free(sj);
        return rc;
    }
    uint64_t i = 0, sum = 0;
    uint64_t prev_q = 0, prev_c = 0, prev_s = 0;
    int have_prev = 0;
    for (uint64_t t = 0; t < m; ++t) {
        uint64_t q = sq[t];
        if (!(have_prev && q == prev_q)) {
            while (i < n && sk[i] < q)
                ++i;
            uint64_t e = i;
            while (e < n && sk[e] == q)
                ++e;
            prev_q = q;
            prev_c = e - i;
            prev_s = i;
            have_prev = 1;
        }
        counts[sj[t]] = (uint32_t)prev_c;
        if (run_start)
            run_start[sj[t]] = (uint32_t)prev_s;
        sum += prev_c;
    }
    *total = sum;
    free(sk);
    free(sq);
    free(sj);
    if (sorted_ids_out)
        *sorted_ids_out = si;
    else
        free(si);
    return ORC_OK;
}

int orc_probe_counts(const void *keys, uint64_t n, const void *queries, uint64_t m,
                     int key_bits, uint32_t *counts, uint64_t *total)
{
    return probe_core(keys, n, queries, m, key_bits, counts, NULL, NULL, total);
}

/* Pairs in canonical order: probe id ascending, then build id ascending.
 * Writes at most `capacity` pairs; returns ORC_ECAPACITY when the total
 * exceeds it (the total is still reported). */
int orc_probe_pairs(const void *keys, uint64_t n, const void *queries, uint64_t m,
                    int key_bits, uint32_t *build_ids, uint32_t *probe_ids,
                    uint64_t capacity, uint64_t *total)
{
    size_t mm = m ? m : 1;
    uint32_t *counts = (uint32_t *)malloc(mm * sizeof(uint32_t));
    uint32_t *start = (uint32_t *)malloc(mm * sizeof(uint32_t));
    uint32_t *sorted_ids = NULL;
    if (!counts || !start) {
        free(counts); free(start);
        return ORC_ENOMEM;
    }
    int rc = probe_core(keys, n, queries, m, key_bits, counts, start, &sorted_ids, total);
    if (rc == ORC_OK) {
        if (*total > capacity) {
            rc = ORC_ECAPACITY;
        } else {
            uint64_t w = 0;
            for (uint64_t j = 0; j < m; ++j)
                for (uint32_t r = 0; r < counts[j]; ++r) {
                    build_ids[w] = sorted_ids[start[j] + r];
                    probe_ids[w] = (uint32_t)j;
                    ++w;
                }
        }
    }
    free(counts);
    free(start);
    free(sorted_ids);
    return rc;
}

/* Brute force: #{i : key[i] == q}, one full scan. */
uint64_t orc_count_one(const void *keys, uint64_t n, int key_bits, uint64_t q)
{
    uint64_t c = 0;
    if (key_bits == 32) {
        const uint32_t *k = (const uint32_t *)keys;
        uint32_t q32 = (uint32_t)q;
        for (uint64_t i = 0; i < n; ++i)
            c += (k[i] == q32);
    } else {
        const uint64_t *k = (const uint64_t *)keys;
        for (uint64_t i = 0; i < n; ++i)
            c += (k[i] == q);
    }
    return c;
}
