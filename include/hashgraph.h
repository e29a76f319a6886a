/*
 * hashgraph.h -- C ABI of libhashgraph.so, the HashGraph hot path on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: O. Green, "HashGraph -- Scalable Hash Tables Using A Sparse Graph
 * Data Structure", arXiv:1907.02900.  A HashGraph is a CSR structure whose
 * vertices are the V hash values and whose edges point back at the N inputs
 * (Sec. 3.1, Fig. 1): an offset array of V+1 entries and an edge array of
 * exactly N entries, each edge holding the input key and its input index.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers (HBM of the current device);
 *     pointers named h_* are host pointers.
 *   - Keys are unsigned integers of key_bits = 32 (uint32_t) or 64 (uint64_t).
 *   - Buckets, offsets, ids and per-query counts are uint32_t, so N, M and V
 *     must be below 2^32.  Totals of pairs are uint64_t.
 *   - Work is enqueued on the given stream and returns before it completes,
 *     except where a host result (h_*) is requested: those calls wait for the
 *     stream.  Passing stream 0 uses the device's null stream.
 *   - The caller owns every buffer it passes.  Inputs are read only while the
 *     enqueued work runs; nothing the caller passes is retained afterwards.
 *   - Tables (hg_table) own their device memory until hg_table_free.  A table
 *     is immutable after its build; probes and intersections may run
 *     concurrently on several streams once the build's stream has passed the
 *     build (for example after hipStreamSynchronize or an event wait).
 *   - No call throws.  Every call returns an hg_status; hg_status_string
 *     gives a message.  Invalid arguments are detected on the host before any
 *     work is enqueued, and then nothing is enqueued and no output is written.
 *   - The library never falls back to the CPU: with no usable gfx950 device
 *     every call that needs one returns HG_ERR_DEVICE.
 */
#ifndef HASHGRAPH_H
#define HASHGRAPH_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hg_status {
    HG_OK = 0,
    HG_ERR_INVALID_ARG = 1, /* bad key_bits, range, size or NULL pointer     */
    HG_ERR_OOM = 2,         /* device allocation failed                      */
    HG_ERR_DEVICE = 3,      /* HIP runtime error or no usable device         */
    HG_ERR_CAPACITY = 4,    /* output capacity too small (total reported)    */
    HG_ERR_MISMATCH = 5,    /* tables built with different hash parameters   */
    HG_ERR_BUDGET = 6,      /* request exceeds the server's memory budget    */
    HG_ERR_NOT_FOUND = 7,   /* unknown table or request handle               */
    HG_ERR_TOO_LARGE = 8    /* size beyond the fixed limit of an entry point */
} hg_status;

/* Build variants (Sec. 3.2 and Sec. 3.3). */
#define HG_VARIANT_AUTO 0 /* V2 */
#define HG_VARIANT_V1 1   /* Alg. 1: global atomic count and atomic scatter  */
#define HG_VARIANT_V2 2   /* Alg. 2: bin partition, then per-bin build       */

typedef struct hg_build_opts {
    int32_t variant;   /* HG_VARIANT_*                                          */
    int32_t stable;    /* 1: ids ascending inside every bucket.  V2 places
                          stably unless any_order is set; V1 places by atomics
                          (order inside a bucket unspecified) and rejects
                          stable=1 with HG_ERR_INVALID_ARG.                     */
    uint32_t bins;     /* V2: number of bins (Alg. 2 "Bins"), rounded so that
                          a bin spans a power-of-two range of buckets; 0 =
                          choose from N and V.                                 */
    uint32_t block;    /* V1: threads per block, 0 = 256                        */
    int32_t no_index;  /* V2 also writes a probe index beside the CSR arrays:
                          one 16-byte entry per bucket holding its length and
                          either all its keys (up to three 32-bit keys) or its
                          start and first key (32-bit keys: with that key's
                          count in the bucket and a 24-bit filter of the
                          bucket's other keys; 64-bit keys: a filter of all
                          keys in place of the first key when the bucket
                          holds two or more), so most probes take one
                          random read.  Buckets of more than 32 entries get a
                          key-run summary instead (distinct keys ascending,
                          each with the end of its group of ids), so probes
                          and intersections of skewed tables cost a binary
                          search instead of a scan.  The whole index is built
                          on the device, in stream order: the build never
                          waits for it.  Its arrays (16 bytes per bucket of
                          the range capacity, and key + 8 bytes per entry of
                          the key capacity for the summary) are allocated by
                          hg_table_create, or by hg_build when it writes the
                          index.  1 = skip the index (probes then read
                          offsets and scan the edge array).  Results are
                          identical either way.  V1 never writes it.         */
    int32_t any_order; /* V2: 1 = the order of ids inside a bucket is
                          unspecified (as in the paper), which lets the
                          partition passes rank without ballots and skips the
                          per-bucket id ordering; offsets, bucket contents as
                          multisets and probe counts are unchanged.  Rejected
                          with stable=1.  0 = stable layout (default).        */
    int32_t v1_plain;  /* V1: 1 = one device-scope atomic per key in the
                          histogram and the scatter, as Alg. 1 prints its
                          loops; 0 (default) = the lanes of a wave whose keys
                          share a bucket are matched by ballots and merged
                          into one atomic (the group's leader adds the
                          group's size and hands out consecutive slots).
                          Results are identical up to the order inside a
                          bucket, which V1 leaves unspecified either way.  */
    uint32_t reserved;
} hg_build_opts;

typedef struct hg_table hg_table; /* opaque; device-resident */

typedef struct hg_table_info {
    const uint32_t *d_offsets; /* V+1 entries, offsets[0]=0, offsets[V]=n      */
    const uint32_t *d_ids;     /* n entries: input index of each edge          */
    const void *d_keys;        /* n keys, bucketed (edge order)                */
    uint64_t n;                /* number of keys (edges)                       */
    uint64_t hash_range;       /* V                                            */
    uint64_t seed;             /* hash seed                                    */
    int32_t key_bits;          /* 32 or 64                                     */
    int32_t variant;           /* variant that built it                        */
    uint64_t device_bytes;     /* device memory the table holds                */
} hg_table_info;

/* Message for a status code; never NULL. */
const char *hg_status_string(hg_status s);

/* Version of this ABI (major*10000 + minor*100 + patch). */
uint32_t hg_version(void);

/* Workspace allocator: lets the caller back the library's temporary device
 * memory with its own allocator, for example PyTorch's caching allocator.
 * Every call that needs temporary device
 * memory -- the build's partition buffers when the table holds no workspace
 * of its own (hg_build; hg_table_create tables never need any), scan
 * partials, the positions of pairs, per-chunk totals -- takes its blocks
 * from alloc_fn(bytes, stream, ctx) and gives each back with
 * free_fn(ptr, stream, ctx) before the call returns, while work it enqueued
 * on that stream may still be reading it.  The allocator must therefore
 * follow stream order: a block freed on a stream is handed out again only to
 * work ordered after the free on that stream (hipMallocAsync and PyTorch's
 * caching allocator do this).  alloc_fn returns NULL when it cannot satisfy
 * the request (the call then fails with HG_ERR_OOM) and must return blocks
 * aligned to 256 bytes (a misaligned block is freed again and the call fails
 * with HG_ERR_INVALID_ARG).  Both functions NULL restore the default,
 * hipMallocAsync / hipFreeAsync; exactly one NULL is HG_ERR_INVALID_ARG.
 * The setting is process-wide and takes effect for calls that start after
 * it; a block already handed out is returned to the functions that gave it.
 * The memory that tables, collections, batch plans and servers keep
 * (hg_table_create, hg_build, hg_collection_build, hg_batch_create,
 * hg_server_create) is their own and does not come from the hook, nor does
 * the per-launch workspace of servers, which counts against their budget.
 * Needs no device. */
typedef void *(*hg_alloc_fn)(size_t bytes, hipStream_t stream, void *ctx);
typedef void (*hg_free_fn)(void *ptr, hipStream_t stream, void *ctx);
hg_status hg_set_allocator(hg_alloc_fn alloc_fn, hg_free_fn free_fn, void *ctx);

/* ------------------------------------------------------------------------
 * Single steps of the path, exposed so that each can be checked alone.
 * ------------------------------------------------------------------------ */

/* Eq. 1 for every key: d_buckets[i] = fmix(d_keys[i] XOR seed) mod V, where
 * fmix is the MurmurHash3 32-bit finaliser for key_bits = 32 (XOR with the
 * low 32 bits of seed) and the 64-bit finaliser for key_bits = 64, and the
 * modulo is exact.  hash_range = V must be in [1, 2^32 - 1].
 * d_keys: n keys; d_buckets: n uint32 (caller-allocated). */
hg_status hg_hash(const void *d_keys, uint64_t n, int key_bits, uint64_t hash_range,
                  uint64_t seed, uint32_t *d_buckets, hipStream_t stream);

/* Alg. 1, loops two and three: d_counts[b] = number of keys whose bucket
 * (as hg_hash) is b, for b in [0, V).  The call zeroes d_counts itself.
 * The atomics of lanes whose keys share a bucket are merged inside each wave
 * (hg_build_opts.v1_plain).  d_counts: V uint32 (caller-allocated). */
hg_status hg_histogram(const void *d_keys, uint64_t n, int key_bits, uint64_t hash_range,
                       uint64_t seed, uint32_t *d_counts, hipStream_t stream);

/* Alg. 1 PrefixSum producing the CSR offset array of Sec. 3.1:
 * d_offsets[0] = 0, d_offsets[b+1] = d_offsets[b] + d_counts[b], for
 * b in [0, V); V+1 outputs.  Sums wrap modulo 2^32.  d_counts: V uint32;
 * d_offsets: V+1 uint32, may not alias d_counts.  V may be 0 (then only
 * d_offsets[0] = 0 is written). */
hg_status hg_exclusive_scan(const uint32_t *d_counts, uint64_t V, uint32_t *d_offsets,
                            hipStream_t stream);

/* ------------------------------------------------------------------------
 * Tables: build (Alg. 1 / Alg. 2), view, free.
 * ------------------------------------------------------------------------ */

/* Build a HashGraph of n keys into a new table.  Equivalent to
 * hg_table_create(n, hash_range, key_bits) followed by hg_table_build.
 * opts may be NULL (defaults).  The device memory of the table and the
 * temporary workspace are allocated by this call (workspace is freed in
 * stream order before the call's work completes). */
hg_status hg_build(const void *d_keys, uint64_t n, int key_bits, uint64_t hash_range,
                   uint64_t seed, const hg_build_opts *opts, hipStream_t stream,
                   hg_table **out);

/* The plan a V2 build (Alg. 2) of n keys over hash_range buckets follows:
 * final bins of 2^bucket_bits consecutive buckets (the paper's Bins, here
 * sized so that a bin's keys fit in LDS), reached by one or two stable
 * partition passes over digits of the bin index, and the workspace the build
 * needs.  bins: as hg_build_opts.bins (0 = the library's choice).  Host only:
 * needs no device.  HG_ERR_INVALID_ARG for key_bits not 32/64, hash_range
 * outside [1, 2^32 - 1], n >= 2^32, bins > hash_range or out NULL. */
typedef struct hg_plan_info {
    uint32_t bucket_bits;     /* k: log2 of the buckets per final bin          */
    uint32_t bins;            /* final bins, ceil(V / 2^k)                     */
    uint32_t passes;          /* partition passes before the per-bin build     */
    uint32_t digit_bits[2];   /* digit width of each pass (0 if unused)        */
    uint32_t tiles[2];        /* partition tiles of each pass (second: bound)  */
    uint32_t tile_keys;       /* keys per partition tile                       */
    uint64_t workspace_bytes; /* device workspace of the build                 */
} hg_plan_info;

hg_status hg_build_plan(uint64_t n, uint64_t hash_range, int key_bits, uint32_t bins,
                        hg_plan_info *out);

/* Autotuner of a single build: chooses the launch parameters of
 * hg_build_opts for these keys by timing candidate builds of them on the
 * stream (into a temporary table it allocates and frees) and returns the
 * fastest in *out.  The semantic fields of base (variant, stable, no_index,
 * any_order; base may be NULL for the defaults) are kept; the tuned fields
 * are, for V2, bins (bins of about 1024, 2048 or -- 32-bit keys -- 4096 keys
 * each, which sets the partition width and the per-bin LDS footprint) and,
 * for V1, block (256, 512 or 1024 threads) and v1_plain (merged or per-key
 * atomics).  The choice is cached in the process, keyed by (ceil log2 n,
 * ceil log2 hash_range, key_bits, the semantic fields, skew class), where
 * the skew class is measured on the first build of these keys (its longest
 * bucket: at most 32, 128 or 512 entries, at most one bin's LDS capacity,
 * or longer); a
 * later call with the same key times only the default build and the cached
 * choice, and returns the latter.  info (may be NULL) reports the times.  Waits for the
 * stream.  Errors as hg_build. */
typedef struct hg_tune_info {
    double ms;           /* time of one build with the returned options        */
    double default_ms;   /* time of one build with the default parameters      */
    uint32_t candidates; /* configurations timed besides the default (0: cached) */
    uint32_t skew_class; /* longest bucket <= 32 entries: 0; <= 128: 1;
                            <= 512: 2; fits a bin's LDS (4608 32-bit / 3072
                            64-bit keys): 3; longer: 4                        */
    uint32_t max_bucket; /* longest bucket of the keys' table                  */
    uint32_t cached;     /* 1: the choice came from the cache                  */
} hg_tune_info;

hg_status hg_build_tune(const void *d_keys, uint64_t n, int key_bits, uint64_t hash_range,
                        uint64_t seed, const hg_build_opts *base, hipStream_t stream,
                        hg_build_opts *out, hg_tune_info *info);

/* Allocate an empty table able to hold up to n_capacity keys and
 * range_capacity buckets, including the workspace a V2 build of that size
 * needs and the probe index with its key-run summary (hg_build_opts.no_index).
 * Later hg_table_build calls of up to those sizes (with the library's choice
 * of bins) allocate nothing and never wait for the device, so a rebuild and
 * the probes after it can be captured into a HIP graph. */
hg_status hg_table_create(uint64_t n_capacity, uint64_t range_capacity, int key_bits,
                          hg_table **out);

/* (Re)build table t from n keys with range V = hash_range and the given seed.
 * Returns HG_ERR_CAPACITY if n or V exceed the table's capacities.  The
 * previous contents are replaced; the caller must not probe t while this
 * build is in flight. */
hg_status hg_table_build(hg_table *t, const void *d_keys, uint64_t n, uint64_t hash_range,
                         uint64_t seed, const hg_build_opts *opts, hipStream_t stream);

/* Describe a table: device pointers to its CSR arrays and its parameters. */
hg_status hg_table_view(const hg_table *t, hg_table_info *info);

/* Copy the table's CSR arrays into caller buffers (device to device, on the
 * stream): d_offsets V+1 uint32, d_ids n uint32, d_keys n keys.  Any of the
 * three may be NULL to skip it.  After hg_table_erase the copy is the
 * compacted CSR of the live entries (their number from hg_table_lengths), in
 * bucket order and, inside a bucket, in the order the build left them. */
hg_status hg_table_export(const hg_table *t, uint32_t *d_offsets, uint32_t *d_ids, void *d_keys,
                          hipStream_t stream);

/* Decremental HashGraph (the per-bucket length array of the paper's
 * conclusion): remove every entry whose key equals one of d_keys[0 .. m)
 * (device array of the table's key width; repeated and absent keys allowed).
 * Bucket h then holds its live entries in [offsets[h], offsets[h] + len[h]);
 * the edge array keeps its size and its order inside each bucket, so a stable
 * table stays stable.  Probes, pairs, intersections and exports see only live
 * entries; a long bucket touched by an erase loses its key runs and is
 * scanned.  Cost: each key scans its bucket, then one pass over the buckets.
 * Requires a V2 table built with the probe index (HG_ERR_INVALID_ARG
 * otherwise); a rebuild starts from a full table again.  h_removed (may be
 * NULL) gets the number of entries removed; waits for the stream.  The first
 * erase allocates the length array and 1 byte per bucket and per entry of
 * scratch flags. */
hg_status hg_table_erase(hg_table *t, const void *d_keys, uint64_t m, uint64_t *h_removed,
                         hipStream_t stream);

/* After an erase: *d_lengths (may be NULL) = device pointer to the per-bucket
 * live lengths (V uint32), or NULL if the table has not been erased since its
 * build; *live (may be NULL) = the number of live entries (n when never
 * erased).  hg_table_view's d_offsets then give each bucket's first slot, its
 * d_ids / d_keys hold stale copies behind each bucket's live entries, and its
 * n stays the number of entries built (the range of ids; size
 * hg_intersect's per-B-entry counts by it). */
hg_status hg_table_lengths(const hg_table *t, const uint32_t **d_lengths, uint64_t *live);

/* Release a table (waits for the device to finish using it).  NULL is a
 * no-op.  Like every call here that frees device memory (hg_collection_free,
 * hg_batch_free, hg_server_destroy), it must not run while a stream of the
 * device is being captured into a graph: the free synchronises, which ends
 * such a capture with an error. */
void hg_table_free(hg_table *t);

/* ------------------------------------------------------------------------
 * Probing (Sec. 3.4).
 * ------------------------------------------------------------------------ */

/* HashGraph-Probe-Standard: for every query j, the number of table entries
 * whose key equals d_queries[j] (all instances, not only the first).
 * d_queries: m keys of the table's key_bits.  d_counts: m uint32 or NULL.
 * h_total: if not NULL, receives the sum of all counts (uint64); this waits
 * for the stream.  At least one of d_counts and h_total must be given.
 * The order the queries are probed in is chosen as by hg_probe_ordered with
 * HG_PROBE_AUTO. */
hg_status hg_probe(const hg_table *t, const void *d_queries, uint64_t m, uint32_t *d_counts,
                   uint64_t *h_total, hipStream_t stream);

/* hg_probe with the probing order given by the caller; counts and total are
 * identical for every order.
 *   HG_PROBE_INPUT_ORDER: every query reads its bucket where it stands (one
 *     random read of the probe index per query, Sec. 3.4).
 *   HG_PROBE_GROUPED: the queries are first partitioned into up to 512
 *     ranges of buckets (with their input positions), probed range by range
 *     with each XCD reading one window of the index at a time, and the
 *     counts are put back in input order.  Needs m * (key_bits / 8 + 8) bytes
 *     of workspace plus 2 KiB per 4096 queries (from the allocator,
 *     hg_set_allocator).
 *   HG_PROBE_GROUPED_UNLESS_SKEWED: the queries' histogram over the ranges
 *     is taken first and, on the device, a range holding more than 8 times
 *     its share of them (skewed queries, whose index lines stay cached
 *     anyway) keeps input order; else grouped.  Workspace as for grouped.
 *   HG_PROBE_AUTO: HG_PROBE_GROUPED_UNLESS_SKEWED when the table has a probe
 *     index, m >= hash_range / 2 and hash_range >= 2^27 (2^26 when only the
 *     total is asked for), the sizes from which grouping measured faster,
 *     and its workspace can be allocated; else input order.
 * Any other order is HG_ERR_INVALID_ARG. */
#define HG_PROBE_AUTO 0
#define HG_PROBE_INPUT_ORDER 1
#define HG_PROBE_GROUPED 2
#define HG_PROBE_GROUPED_UNLESS_SKEWED 3
hg_status hg_probe_ordered(const hg_table *t, const void *d_queries, uint64_t m,
                           uint32_t *d_counts, uint64_t *h_total, int32_t order,
                           hipStream_t stream);

/* The matching pairs themselves: d_build_ids[p], d_probe_ids[p] for p below
 * the total, grouped by probe id ascending; inside one probe id the build
 * ids follow the table's bucket order (ascending for stable tables).
 * Always writes *h_total (required) and waits for the stream.  If the total
 * exceeds capacity, nothing is written to the pair arrays and
 * HG_ERR_CAPACITY is returned. */
hg_status hg_probe_pairs(const hg_table *t, const void *d_queries, uint64_t m,
                         uint32_t *d_build_ids, uint32_t *d_probe_ids, uint64_t capacity,
                         uint64_t *h_total, hipStream_t stream);

/* hg_probe_pairs for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, outputs, order and errors as hg_probe_pairs, but the
 * call's workspace (per-query counts, their 64-bit exclusive scan and the
 * scan's partials) lives in a fixed device array inside the library instead
 * of being allocated: the call makes no allocation of any kind.  That array
 * (52 MiB) exists once per device the library runs on and stays held until
 * the process ends.  Limit: m <= HG_NOALLOC_MAX_QUERIES (2^22); larger m
 * returns HG_ERR_TOO_LARGE before anything is enqueued.  Every call on a
 * device shares that device's array and the array keeps what the last call
 * left in it (each call writes every byte it reads first, so nothing needs
 * clearing): calls that overlap on one device -- from two host threads, or
 * on two streams -- race and give wrong pairs; serialise them.  Waits for
 * the stream (it returns the total). */
#define HG_NOALLOC_MAX_QUERIES (1u << 22)
hg_status hg_probe_pairs_noalloc(const hg_table *t, const void *d_queries, uint64_t m,
                                 uint32_t *d_build_ids, uint32_t *d_probe_ids,
                                 uint64_t capacity, uint64_t *h_total, hipStream_t stream);

/* HashGraph-Probe-New (Alg. 3): bucket-wise intersection of tables a and b,
 * which must share key_bits, hash_range and seed (else HG_ERR_MISMATCH).
 * d_counts_b: if not NULL, n_b uint32, indexed by b's INPUT index j: the
 * number of entries of a whose key equals b's key j.  d_a_ids / d_b_ids with
 * capacity > 0: the matching (a input index, b input index) pairs, grouped
 * by b's edge order.  h_total: if not NULL receives the number of pairs and
 * the call waits for the stream; required when capacity > 0.  Returns
 * HG_ERR_CAPACITY (pairs not written, total reported) if the total exceeds
 * a non-zero capacity. */
hg_status hg_intersect(const hg_table *a, const hg_table *b, uint32_t *d_counts_b,
                       uint32_t *d_a_ids, uint32_t *d_b_ids, uint64_t capacity,
                       uint64_t *h_total, hipStream_t stream);

/* Alg. 3's counts in the order it produces them: d_counts_edges[p] (n_b
 * uint32, may be NULL) = the number of entries of a whose key equals the key
 * at b's edge position p (b's input index of that entry is d_ids[p] of
 * hg_table_view; after an erase, stale positions get 0).  Unlike
 * hg_intersect's per-input counts, nothing is scattered: every write is
 * sequential.  h_total (may be NULL; waits for the stream) receives the join
 * size.  Same requirements and errors as hg_intersect. */
hg_status hg_intersect_edges(const hg_table *a, const hg_table *b, uint32_t *d_counts_edges,
                             uint64_t *h_total, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Collections: build once, intersect many (Sec. 3.4).  Probe-New pays for a
 * second table; in sparse products that cost is amortised, because the table
 * of every row or column is built once and takes part in many
 * intersections.  A collection holds S key sets, each with its own table;
 * hg_collection_intersect then counts the matches of many (set, set) pairs.
 *
 * Layout.  Set s is d_keys[set_offsets[s] .. set_offsets[s+1]) with n_s keys.
 * Its hash range V_s is a power of two: the smallest one >= max(n_s, 1),
 * times 2^range_shift, clamped to [1, 2^31]; its buckets use the hash of
 * Eq. 1 (fmix32 / fmix64 of key ^ seed, low bits).  The tables are
 * concatenated: set s owns buckets [bucket_base[s], bucket_base[s+1]) of one
 * offsets array, whose entries are absolute positions in the shared ids and
 * keys arrays, and its entries fill [set_offsets[s], set_offsets[s+1]) of
 * them, grouped by bucket with ids ascending inside a bucket.  Ids are
 * positions in the concatenated input.  Set s's table is thus the stable
 * HashGraph of its keys with range V_s (Alg. 2), its offsets and ids shifted
 * by set_offsets[s].
 * ------------------------------------------------------------------------ */

typedef struct hg_collection hg_collection; /* opaque; owns its device arrays */

typedef struct hg_collection_info {
    uint32_t sets;                 /* S                                          */
    int32_t key_bits;              /* 32 or 64                                   */
    uint64_t seed;                 /* hash seed                                  */
    int32_t range_shift;           /* see the layout above                       */
    uint32_t reserved;
    uint64_t n;                    /* entries, set_offsets[S]                    */
    uint64_t buckets;              /* sum of V_s                                 */
    uint64_t heavy_keys;           /* entries of the sets built by the sort path */
    uint64_t bytes;                /* device bytes the collection holds          */
    const uint32_t *d_set_offsets; /* S + 1 (a copy of the input's)              */
    const uint64_t *d_bucket_base; /* S + 2; bucket_base[S] = bucket_base[S+1] = buckets */
    const uint32_t *d_offsets;     /* buckets + 1                                */
    const uint32_t *d_ids;         /* n                                          */
    const void *d_keys;            /* n keys of key_bits                         */
} hg_collection_info;

/* Build every set's table.  d_keys: set_offsets[S] device keys of key_bits;
 * d_set_offsets: S + 1 device uint32, set_offsets[0] = 0, non-decreasing
 * (checked on the device: HG_ERR_INVALID_ARG otherwise, nothing kept).
 * range_shift in [-31, 31]; HG_ERR_INVALID_ARG if the total of the V_s
 * reaches 2^32 - 1.  Sets of a few thousand keys or fewer are built in LDS,
 * several per workgroup; heavier sets together by one radix sort.  Allocates
 * the collection (4 (buckets + 1) + (4 + key_bits / 8) n + 12 (S + 2) bytes)
 * and workspace; waits for the stream.  The input may be freed afterwards. */
hg_status hg_collection_build(const void *d_keys, const uint32_t *d_set_offsets, uint32_t sets,
                              int key_bits, uint64_t seed, int32_t range_shift,
                              hg_collection **out, hipStream_t stream);

/* Describe a collection: its sizes and device pointers to its arrays. */
hg_status hg_collection_view(const hg_collection *c, hg_collection_info *info);

/* Copy the collection's arrays into caller buffers (device to device, on the
 * stream): d_bucket_base S + 2 uint64, d_offsets buckets + 1 uint32, d_ids n
 * uint32, d_keys n keys.  Any of them may be NULL to skip it. */
hg_status hg_collection_export(const hg_collection *c, uint64_t *d_bucket_base,
                               uint32_t *d_offsets, uint32_t *d_ids, void *d_keys,
                               hipStream_t stream);

/* Match counts of set pairs: for q < pairs, with (i, j) = (d_pairs[2q],
 * d_pairs[2q+1]) naming set i of a and set j of b, d_counts[q] (uint64, may
 * be NULL) = the number of (x, y) with x an entry of a's set i, y an entry of
 * b's set j and equal keys (the join size; for sets without repeated keys,
 * the size of their intersection).  The smaller set of each pair is walked in
 * its table's order and looked up in the other's buckets.  a and b may be the
 * same collection; they must share key_bits and seed (HG_ERR_MISMATCH).  An
 * index out of range gives HG_ERR_INVALID_ARG (counts then unspecified).
 * h_total (may be NULL) receives the sum over all pairs.  Waits for the
 * stream (the pair work is sized on the host). */
hg_status hg_collection_intersect(const hg_collection *a, const hg_collection *b,
                                  const uint32_t *d_pairs, uint64_t pairs, uint64_t *d_counts,
                                  uint64_t *h_total, hipStream_t stream);

/* Release a collection (waits for the device).  NULL is a no-op. */
void hg_collection_free(hg_collection *c);

/* ------------------------------------------------------------------------
 * Batched build + probe: many independent tables in one hipGraph launch.
 * Each table is built exactly as hg_build builds it with the V2 variant (the
 * stable layout of Alg. 2) into the caller's output arrays, then probed as
 * hg_probe probes it.  Intended for thousands of small and medium tables.
 * ------------------------------------------------------------------------ */

typedef struct hg_batch_item {
    const void *d_keys;    /* n keys of the batch's key width                   */
    uint64_t n;            /* < 2^32                                            */
    uint64_t hash_range;   /* V in [1, 2^32 - 1]                                */
    uint64_t seed;         /* hash seed                                         */
    const void *d_queries; /* m queries (may be NULL when m == 0)               */
    uint64_t m;            /* < 2^32                                            */
    uint32_t *d_offsets;   /* out: V+1 CSR offsets                              */
    uint32_t *d_ids;       /* out: n input indices, bucketed                    */
    void *d_ekeys;         /* out: n keys, bucketed                             */
    uint32_t *d_counts;    /* out: m per-query match counts (NULL when m == 0)  */
} hg_batch_item;

typedef struct hg_batch_opts {
    uint32_t autotune;      /* 1 (default when opts is NULL): choose every
                               launch parameter left at 0 below by timing
                               candidate graphs on this batch, one dimension
                               at a time (bin target, then partition keys per
                               thread, then probe workgroup shape), keeping
                               the fastest; the choice is cached per batch
                               shape (tables, total keys, total queries, key
                               width, layout).  0: parameters left at 0 take
                               their defaults (2048, 16, 256 x 4).          */
    uint32_t bin_target;    /* keys per final bin of the partitioned tables
                               (sets the partition width: the number of
                               digits a tile scatters to); 0 = tune/default.
                               Candidates: 1024, 2048 and, for 32-bit keys,
                               4096.                                         */
    uint32_t any_order;     /* 1: order of ids inside a bucket unspecified (as
                               hg_build_opts.any_order); 0: stable layout    */
    uint32_t part_items;    /* keys per thread of a partition tile (256
                               threads): 8 or 16; 0 = tune/default (16).     */
    uint32_t probe_threads; /* probe workgroup shape, threads x queries per  */
    uint32_t probe_items;   /* thread: 256x4, 256x8, 512x2 or 128x8; both 0 =
                               tune/default (256x4).  Other values, or one of
                               the two 0, are HG_ERR_INVALID_ARG.            */
    uint32_t reserved[2];
} hg_batch_opts;

typedef struct hg_batch hg_batch; /* opaque plan: device descriptors, workspace
                                     and the captured graph */

/* Plan a batch of `count` tables (host array of descriptors; every pointer in
 * it is a device pointer).  Uploads descriptors, allocates the shared
 * workspace, autotunes (which runs the batch a few times on the device, so
 * the output buffers are written) and captures the run into a hipGraph.  The
 * plan keeps the pointers: the caller's buffers must stay allocated until
 * hg_batch_free; their contents may change between runs.  Waits for the
 * device.  Tables with a hash range above 2^23 (2048 bins of 4096 buckets;
 * about 2^23 keys at load 1) are rejected with HG_ERR_INVALID_ARG: build those with
 * hg_build. */
hg_status hg_batch_create(const hg_batch_item *items, uint32_t count, int key_bits,
                          const hg_batch_opts *opts, hg_batch **out);

/* Build and probe every table of the batch: one graph launch on `stream`. */
hg_status hg_batch_run(hg_batch *b, hipStream_t stream);

/* The chosen keys-per-bin target and the workspace the plan holds. */
hg_status hg_batch_info(const hg_batch *b, uint32_t *bin_target, uint64_t *workspace_bytes);

/* The launch configuration the plan runs with (every tunable field set,
 * autotune = 0): passing it to hg_batch_create plans the same graph without
 * tuning. */
hg_status hg_batch_config(const hg_batch *b, hg_batch_opts *out);

/* Release a plan (waits for the device).  NULL is a no-op. */
void hg_batch_free(hg_batch *b);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 * Build and probe requests are queued and return at once; a host thread in
 * the library admits them onto several HIP streams as launch slots and
 * memory allow, so the work of different requests overlaps on the device.
 * Small requests pending at the same time are merged into one launch of the
 * batched kernels.  Tables stay resident on the device under a byte budget
 * (resident tables plus in-flight workspace); when a request does not fit,
 * the least recently used tables that no pending or running request needs
 * are evicted.  Results are the same as hg_build (V2) / hg_probe give.
 * Latency is measured from submission to the moment the loop observes the
 * request's completion (resolution about 20 microseconds).
 * ------------------------------------------------------------------------ */

typedef struct hg_server hg_server;

typedef struct hg_server_opts {
    uint64_t budget_bytes; /* device bytes for resident tables + in-flight work;
                              0 = 64 GiB                                       */
    uint32_t streams;      /* HIP streams, default priority; 0 = 4 (max 16)    */
    uint32_t max_inflight; /* launches in flight at once; 0 = 8 (max 256)      */
    uint32_t merge_max;    /* most requests merged into one launch; 0 = 64,
                              1 = never merge                                  */
    uint32_t merge_keys;   /* requests of at most this many keys or queries
                              may be merged; 0 = 2^18.  Tables built in a
                              merged launch carry no probe index (their
                              probes read offsets and scan)                  */
    uint32_t workers;      /* host threads that launch the device work, each
                              on its own share of the streams; 0 = 2 (or 1
                              with one stream); at most 8 and at most
                              `streams`                                      */
    uint32_t reserved[3];
} hg_server_opts;

typedef struct hg_server_stats {
    uint64_t completed, failed, rejected, evictions;
    uint64_t launches;        /* device launches issued                        */
    uint64_t merged_requests; /* requests that ran inside merged launches      */
    uint64_t keys;            /* keys + queries of completed requests          */
    double p50_ms, p99_ms, mean_ms, max_ms; /* submission -> completion, over
                                               the last 2^20 completed requests
                                               since the last reset           */
    double busy_s;            /* first submission -> last completion           */
    uint64_t resident_bytes, peak_bytes;
    uint32_t resident_tables;
    uint32_t held_requests;   /* request records not yet released (see
                                 hg_server_wait / hg_server_drain)             */
} hg_server_stats;

/* Start a server on the current device (opts may be NULL). */
hg_status hg_server_create(const hg_server_opts *opts, hg_server **out);

/* Queue a build of n keys (device pointer, must stay valid until the request
 * completes).  *table_id names the table for later probes; *request_id (may
 * be NULL) can be waited on.  A table larger than the whole budget fails with
 * HG_ERR_BUDGET (reported by hg_server_wait).  A request submitted with
 * request_id NULL keeps no record after it completes; otherwise its record
 * (status) is kept until hg_server_wait or hg_server_drain releases it. */
hg_status hg_server_submit_build(hg_server *s, const void *d_keys, uint64_t n, int key_bits,
                                 uint64_t hash_range, uint64_t seed, uint64_t *table_id,
                                 uint64_t *request_id);

/* Queue a probe of m queries against a table; per-query counts go to
 * d_counts (device, m uint32).  The table is pinned against eviction from
 * now until this probe completes.  HG_ERR_NOT_FOUND if the table is unknown,
 * was evicted or failed to build. */
hg_status hg_server_submit_probe(hg_server *s, uint64_t table_id, const void *d_queries,
                                 uint64_t m, uint32_t *d_counts, uint64_t *request_id);

/* Block until a request has completed; *result (may be NULL) receives its
 * status.  The request's record is then released: a second wait on the same
 * id (or a wait after hg_server_drain) returns HG_ERR_NOT_FOUND. */
hg_status hg_server_wait(hg_server *s, uint64_t request_id, hg_status *result);

/* Block until every submitted request has completed, then release the
 * records of all completed requests. */
hg_status hg_server_drain(hg_server *s);

/* The CSR arrays of a resident, built table (device pointers owned by the
 * server, valid until the table is evicted or the server destroyed). */
hg_status hg_server_table(hg_server *s, uint64_t table_id, hg_table_info *info);

/* Copy a resident, built table's CSR arrays into caller buffers (device to
 * device on `stream`; any pointer may be NULL).  HG_ERR_NOT_FOUND if the
 * table is not resident.  The copy is ordered after the table's build and
 * the call waits for it. */
hg_status hg_server_export(hg_server *s, uint64_t table_id, uint32_t *d_offsets, uint32_t *d_ids,
                           void *d_keys, hipStream_t stream);

hg_status hg_server_stats_get(hg_server *s, hg_server_stats *out);
hg_status hg_server_reset_stats(hg_server *s);

/* Finish all queued work, free every table and stop the loop. */
void hg_server_destroy(hg_server *s);

/* ------------------------------------------------------------------------
 * Measurement: per-kernel timing with HIP events.
 * ------------------------------------------------------------------------ */

/* Turn event timing of the library's kernel launches on (1) or off (0).
 * While on, each launch records a HIP event before and after itself on the
 * stream it runs on (a small overhead per launch). */
hg_status hg_profile_enable(int on);

/* Drop all recorded launches (waits for their events). */
hg_status hg_profile_reset(void);

/* Aggregate the recorded launches by kernel name (waits for their events);
 * *count receives the number of distinct kernels, indexable below. */
hg_status hg_profile_count(uint32_t *count);

/* Name (NUL-terminated, truncated to name_cap), launch count and summed
 * duration in milliseconds of aggregated kernel `index`. */
hg_status hg_profile_get(uint32_t index, char *name, uint32_t name_cap, uint64_t *launches,
                         double *total_ms);

/* Random-transaction micro-roofline: the ceiling of random-access kernels
 * (the probe makes one random 16-byte read per query, V1 one random atomic
 * add per key).  Allocates a zeroed buffer of footprint_bytes (a power of two,
 * >= 4096), runs `accesses` independent random accesses of the given kind
 * over it once to warm up and once timed (HIP events on `stream`), frees the
 * buffer and stores the timed run's milliseconds in *h_ms.  Waits for the
 * device. */
enum {
    HG_MICRO_READ4 = 0,   /* random 4-byte loads           */
    HG_MICRO_READ16 = 1,  /* random 16-byte (uint4) loads  */
    HG_MICRO_ATOMIC4 = 2  /* random 4-byte atomic adds     */
};
hg_status hg_random_access_rate(int kind, uint64_t footprint_bytes, uint64_t accesses,
                                double *h_ms, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HASHGRAPH_H */
