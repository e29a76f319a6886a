/*
 * Multi-core variant of the CPU oracle (OpenMP), for the CPU baseline.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Same status as hg_oracle.c: only
 * the test suite and the benchmark's CPU-baseline leg load it, and it shares
 * no source with the HIP library.
 *
 * It computes the same definitions as the sequential oracle, on all host
 * cores, and its outputs are identical to it bit for bit (pinned in
 * tests/test_oracle_pins.py):
 *   orc_build_omp         the stable HashGraph table (Sec. 3.1, Alg. 1/2:
 *                         bucket of Eq. 1 for every key, offsets = exclusive
 *                         prefix of the bucket counts, ids ascending inside
 *                         each bucket).  The stable table is the input ids
 *                         stably sorted by bucket, so it is computed as a
 *                         stable LSD radix sort of (bucket, id) pairs; the
 *                         offsets are read off the sorted buckets.
 *   orc_probe_counts_omp  count[j] = #{i : key[i] == query[j]} (Sec. 3.4
 *                         Probe-Standard reports every instance), by sorting
 *                         both sides by key and merging, as orc_probe_counts.
 *
 * The radix sort: per pass, each thread counts the digits of its contiguous
 * chunk, the (digit, thread) counts are prefix-summed digit-major, and each
 * thread scatters its chunk in order, which keeps the sort stable.
 *
 * Return codes as hg_oracle.c.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2

uint32_t orc_bucket_one(uint64_t key, int key_bits, uint64_t V, uint64_t seed);

/* threads the parallel regions use */
int orc_omp_threads(void) { return omp_get_max_threads(); }

/* Stable LSD radix sort of n (key, val) pairs by the low `bits` bits of key,
 * 8 bits per pass.  k/v hold the input; tk/tv are scratch of the same size.
 * On return the sorted pairs are in *ko/*vo (one of the two buffers). */
static int radix_pairs(uint64_t *k, uint32_t *v, uint64_t *tk, uint32_t *tv, uint64_t n,
                       int bits, uint64_t **ko, uint32_t **vo)
{
    const int T = omp_get_max_threads();
    uint64_t *cnt = (uint64_t *)malloc((size_t)T * 256 * sizeof(uint64_t));
    if (!cnt)
        return ORC_ENOMEM;
    for (int shift = 0; shift < bits; shift += 8) {
        memset(cnt, 0, (size_t)T * 256 * sizeof(uint64_t));
#pragma omp parallel num_threads(T)
        {
            const int t = omp_get_thread_num();
            const uint64_t lo = n * (uint64_t)t / (uint64_t)T;
            const uint64_t hi = n * (uint64_t)(t + 1) / (uint64_t)T;
            uint64_t *c = cnt + (size_t)t * 256;
            for (uint64_t i = lo; i < hi; ++i)
                c[(k[i] >> shift) & 0xff] += 1;
#pragma omp barrier
#pragma omp single
            {
                uint64_t run = 0;
                for (int d = 0; d < 256; ++d)
                    for (int u = 0; u < T; ++u) {
                        uint64_t x = cnt[(size_t)u * 256 + d];
                        cnt[(size_t)u * 256 + d] = run;
                        run += x;
                    }
            }
            for (uint64_t i = lo; i < hi; ++i) {
                uint64_t p = c[(k[i] >> shift) & 0xff]++;
                tk[p] = k[i];
                tv[p] = v[i];
            }
        }
        uint64_t *sk = k; k = tk; tk = sk;
        uint32_t *sv = v; v = tv; tv = sv;
    }
    free(cnt);
    *ko = k;
    *vo = v;
    return ORC_OK;
}

static int bits_for(uint64_t V)
{
    int b = 0;
    while (b < 64 && (V - 1) >> b)
        ++b;
    return b;
}

int orc_build_omp(const void *keys, uint64_t n, int key_bits, uint64_t V, uint64_t seed,
                  uint32_t *offsets, uint32_t *ids, void *ekeys)
{
    if (!(key_bits == 32 || key_bits == 64) || V < 1 || V > 0xffffffffull ||
        n > 0xffffffffull)
        return ORC_EINVAL;
    size_t nn = n ? n : 1;
    uint64_t *hk = (uint64_t *)malloc(nn * sizeof(uint64_t));
    uint64_t *tk = (uint64_t *)malloc(nn * sizeof(uint64_t));
    uint32_t *iv = (uint32_t *)malloc(nn * sizeof(uint32_t));
    uint32_t *tv = (uint32_t *)malloc(nn * sizeof(uint32_t));
    int rc = ORC_ENOMEM;
    if (hk && tk && iv && tv) {
        const uint32_t *k32 = (const uint32_t *)keys;
        const uint64_t *k64 = (const uint64_t *)keys;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)n; ++i) {
            uint64_t key = key_bits == 32 ? (uint64_t)k32[i] : k64[i];
            hk[i] = orc_bucket_one(key, key_bits, V, seed);
            iv[i] = (uint32_t)i;
        }
        uint64_t *sh;
        uint32_t *si;
        rc = radix_pairs(hk, iv, tk, tv, n, bits_for(V), &sh, &si);
        if (rc == ORC_OK) {
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < (int64_t)n; ++p) {
                uint32_t i = si[p];
                ids[p] = i;
                if (key_bits == 32)
                    ((uint32_t *)ekeys)[p] = k32[i];
                else
                    ((uint64_t *)ekeys)[p] = k64[i];
            }
            /* offsets[b] = number of entries with bucket < b: position p
             * (0 <= p <= n) is the offset of every bucket in
             * (bucket[p-1], bucket[p]], with bucket[-1] = -1 and bucket[n] = V */
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p <= (int64_t)n; ++p) {
                uint64_t from = p ? sh[p - 1] + 1 : 0;
                uint64_t to = p < (int64_t)n ? sh[p] : V;
                for (uint64_t b = from; b <= to; ++b)
                    offsets[b] = (uint32_t)p;
            }
        }
    }
    free(hk);
    free(tk);
    free(iv);
    free(tv);
    return rc;
}

/* keys widened to 64 bits, sorted with their input index */
static int sorted_side(const void *keys, uint64_t n, int key_bits, uint64_t **bufs,
                       uint32_t **ibufs, uint64_t **ko, uint32_t **vo)
{
    size_t nn = n ? n : 1;
    bufs[0] = (uint64_t *)malloc(nn * sizeof(uint64_t));
    bufs[1] = (uint64_t *)malloc(nn * sizeof(uint64_t));
    ibufs[0] = (uint32_t *)malloc(nn * sizeof(uint32_t));
    ibufs[1] = (uint32_t *)malloc(nn * sizeof(uint32_t));
    if (!bufs[0] || !bufs[1] || !ibufs[0] || !ibufs[1])
        return ORC_ENOMEM;
    const uint32_t *k32 = (const uint32_t *)keys;
    const uint64_t *k64 = (const uint64_t *)keys;
    uint64_t *k = bufs[0];
    uint32_t *v = ibufs[0];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        k[i] = key_bits == 32 ? (uint64_t)k32[i] : k64[i];
        v[i] = (uint32_t)i;
    }
    return radix_pairs(bufs[0], ibufs[0], bufs[1], ibufs[1], n, key_bits, ko, vo);
}

/* first index in sorted a[0..n) whose value is >= x */
static uint64_t lower_bound(const uint64_t *a, uint64_t n, uint64_t x)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

int orc_probe_counts_omp(const void *keys, uint64_t n, const void *queries, uint64_t m,
                         int key_bits, uint32_t *counts, uint64_t *total)
{
    if (!(key_bits == 32 || key_bits == 64) || n > 0xffffffffull || m > 0xffffffffull)
        return ORC_EINVAL;
    uint64_t *kb[2] = {0, 0}, *qb[2] = {0, 0};
    uint32_t *ki[2] = {0, 0}, *qi[2] = {0, 0};
    uint64_t *sk, *sq;
    uint32_t *si, *sj;
    int rc = sorted_side(keys, n, key_bits, kb, ki, &sk, &si);
    if (rc == ORC_OK)
        rc = sorted_side(queries, m, key_bits, qb, qi, &sq, &sj);
    uint64_t sum = 0;
    if (rc == ORC_OK) {
        const int T = omp_get_max_threads();
#pragma omp parallel num_threads(T) reduction(+ : sum)
        {
            const int t = omp_get_thread_num();
            const uint64_t lo = m * (uint64_t)t / (uint64_t)T;
            const uint64_t hi = m * (uint64_t)(t + 1) / (uint64_t)T;
            uint64_t i = lo < hi ? lower_bound(sk, n, sq[lo]) : 0;
            for (uint64_t u = lo; u < hi; ++u) {
                uint64_t q = sq[u];
                while (i < n && sk[i] < q)
                    ++i;
                uint64_t e = i;
                while (e < n && sk[e] == q)
                    ++e;
                counts[sj[u]] = (uint32_t)(e - i);
                sum += e - i;
            }
        }
        *total = sum;
    }
    for (int b = 0; b < 2; ++b) {
        free(kb[b]);
        free(qb[b]);
        free(ki[b]);
        free(qi[b]);
    }
    return rc;
}
