/*
 * hg.h -- C ABI of the HashGraph build and probe on one MI355X (gfx950).
 *
 * The method (Tripathy & Green, "Scalable Hash Table for NUMA Systems",
 * arXiv 2104.00792) stores a static hash table as a CSR graph: an offset
 * array over the hash range and a key array grouped by hash value
 * (Sec. 3.1, "Compressed-Sparse Row" and "Building HashGraph").  The table is
 * built by hashing, counting keys per hash value, an exclusive prefix sum and
 * a scatter (Algorithm 1).  The multi-GPU build first splits the keys into
 * hash-range partitions by count, prefix sum and scatter (Algorithm 2,
 * Phase 2); this library performs one GPU's share of it: the split, then a
 * local table per partition, with no cross-GPU exchange.
 *
 * Conventions shared by every entry point
 *   - Pointers named d_* are device pointers on the current HIP device; the
 *     others are host pointers.  Inputs are never modified.
 *   - Work is enqueued on `stream` and is asynchronous unless stated.  The
 *     caller keeps inputs and outputs alive until the stream reaches them.
 *   - Argument errors are detected on the host before anything is enqueued
 *     and return HG_ERR_INVALID_ARG or HG_ERR_UNSUPPORTED; outputs are then
 *     untouched.  HIP failures return HG_ERR_HIP (hg_last_error() holds the
 *     message).  On any error nothing is leaked.
 *   - Keys are unsigned 32- or 64-bit integers; every value is a legal key
 *     (no sentinel).  n and q are below 2^32 per call.
 *   - hash(k) is the MurmurHash3 finalizer of the key value: fmix32 for
 *     32-bit keys, fmix64 for 64-bit keys (Sec. 4.2 names Murmur).
 *   - Partition of a key: the top log2(P) bits of hash(k).
 *   - Table size of partition p: V_p = max(1, floor(n_p * ratio_num /
 *     ratio_den)), i.e. V = N / C with load factor C (Sec. 2); a plain table
 *     (P == 1) may instead fix V with num_buckets.
 *   - Bucket of a key: hash(k) mod V_p (Algorithm 1, first loop; a true
 *     remainder).  Global bucket g = bucket_base[p] + bucket, where
 *     bucket_base is the exclusive prefix sum of V_p, so the P local tables
 *     form one CSR over sum(V_p) buckets.
 *   - The library is thread-safe across distinct tables and streams.
 */
#ifndef HG_H
#define HG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hg_status {
  HG_OK = 0,
  HG_ERR_INVALID_ARG = 1,   /* null pointer, n >= 2^32, V = 0, bad P ...   */
  HG_ERR_OUT_OF_MEMORY = 2, /* device allocation failed                     */
  HG_ERR_HIP = 3,           /* a HIP call failed (see hg_last_error)        */
  HG_ERR_UNSUPPORTED = 4    /* legal request outside what is implemented    */
} hg_status;

typedef enum hg_key_type { HG_KEY_U32 = 0, HG_KEY_U64 = 1 } hg_key_type;

/* Build options.
 *   P            number of hash-range partitions: 1 (plain table) or a power
 *                of two up to 256 (Algorithm 2, Phase 2 with equal ranges).
 *   ratio_num/ratio_den
 *                table ratio 1/C: V_p = max(1, floor(n_p * num / den)).
 *                Both nonzero unless num_buckets is used.
 *   num_buckets  if nonzero and P == 1: the bucket count V itself
 *                (1 <= V <= 2^32 - 2); otherwise ignored.
 *   log2_subbin  sorted build: sub-bins of 2^log2_subbin buckets (10..13),
 *                which sets the keys each workgroup of the LDS build takes;
 *                0 lets the library choose: about 2^13 keys per sub-bin,
 *                so tables with many keys per bucket (the duplicate study
 *                of Sec. 5.4) get sub-bins of fewer than 2^10 buckets, a
 *                size this knob does not offer.
 *   split_bits   sorted build: at most 2^split_bits level-2 digits per
 *                level-1 segment (7..10); 0 lets the library choose.
 * The last two change speed only, never the table; a table keeps them for
 * its probes.  The total bucket count sum(V_p) must stay below 2^32 - 1
 * (32-bit offsets, Sec. 4.3 keeps the table size 32-bit). */
typedef struct hg_build_opts {
  uint32_t P;
  uint32_t ratio_num;
  uint32_t ratio_den;
  uint32_t flags;     /* HG_BUILD_* below; 0 lets the library choose */
  uint64_t num_buckets;
  uint32_t log2_subbin;
  uint32_t split_bits;
} hg_build_opts;

/* Build strategies (same table, different kernels).  ATOMIC: histogram and
 * scatter with global atomics, as written in Algorithm 1 (fast while the
 * counters fit in cache).  SORTED: two splits down to sub-bins of at most
 * 2^13 buckets, then histogram, scan and scatter inside LDS (the paper's
 * local binning of Sec. 3.2 carried down to LDS size). */
#define HG_BUILD_ATOMIC 1u
#define HG_BUILD_SORTED 2u

/* Probe strategies for hg_count_ex / hg_query_ex.  DIRECT: each query reads
 * its bucket's offsets and keys where they lie.  SORTED: queries take the
 * table's two splits, are counted against LDS-resident windows of the table,
 * and return to input order by two gathers. */
#define HG_PROBE_DIRECT 1u
#define HG_PROBE_SORTED 2u

/* Opaque table.  It owns device memory for:
 *   keys[n]            keys grouped by global bucket (order inside a bucket
 *                      is unspecified, as with the atomics of Algorithm 1),
 *   offsets[B + 1]     CSR offsets, B = sum(V_p): bucket g holds
 *                      keys[offsets[g] .. offsets[g+1]), offsets[B] = n,
 *   part_offsets[P+1]  first key of each partition, part_offsets[P] = n,
 *   bucket_base[P+1]   first global bucket of each partition. */
typedef struct hg_table hg_table;

/* Host-side description of a built table (hg_table_info). */
typedef struct hg_table_desc {
  uint64_t n;             /* keys in the table                              */
  uint64_t num_buckets;   /* B = sum(V_p)                                   */
  uint32_t P;             /* partitions                                     */
  uint32_t key_type;      /* hg_key_type                                    */
  const void* d_keys;     /* n keys                                         */
  const uint32_t* d_offsets;      /* B + 1                                  */
  const uint32_t* d_part_offsets; /* P + 1                                  */
  const uint32_t* d_bucket_base;  /* P + 1                                  */
  uint32_t probe_count_bytes;     /* width of the counts that a sorted probe
                                     passes between its kernels: 1 when no
                                     bucket holds more than 64 keys (no key
                                     then occurs more often), else 4        */
  uint32_t reserved;
} hg_table_desc;

/* hg_build -- build a static table from all n keys (Algorithm 1; with
 * P > 1, Algorithm 2 Phase 2 then Phase 4 on this GPU's keys).
 *   d_keys  n keys of type kt (read only; the table keeps its own copy).
 *   opts    build options (required).
 *   out     receives the new table; set only on HG_OK.
 * Allocates the table and temporary workspace from the library's block
 * cache (or the allocator of hg_set_allocator); the call does not
 * synchronize (only a cache miss, served by hipMalloc, may wait).  n = 0 builds an empty table (every bucket empty, every
 * count 0).  Errors: HG_ERR_INVALID_ARG for
 * null d_keys with n > 0, null opts/out, n >= 2^32, P not a power of two,
 * a zero ratio without num_buckets, too many buckets, unknown flags, or
 * log2_subbin / split_bits outside their ranges; HG_ERR_UNSUPPORTED for
 * P > 256. */
hg_status hg_build(const void* d_keys, uint64_t n, hg_key_type kt,
                   const hg_build_opts* opts, hipStream_t stream,
                   hg_table** out);

/* hg_build_like -- a HashGraph of n keys (the query set) with the layout of
 * `table`: the same partitions, table sizes V_p and bucket bases, so that
 * bucket g of both tables holds exactly the keys that hash to g (Sec. 3.3,
 * "Querying": the query set gets its own HashGraph over the same hash
 * values).  The keys have the table's key type.  Errors: as hg_build, plus
 * HG_ERR_INVALID_ARG for a null or batched table. */
hg_status hg_build_like(const hg_table* table, const void* d_keys, uint64_t n,
                        hipStream_t stream, hg_table** out);

/* hg_intersect -- the per-bucket list intersections of Sec. 3.3: for every
 * position j of the query table's key array (bucket order, see
 * hg_table_info), d_counts[j] = number of keys of `table` equal to that
 * query key; both lists are the same bucket's.  `queries` must come from
 * hg_build_like(table, ...).  d_counts: queries' n uint32.  Errors:
 * HG_ERR_INVALID_ARG for null tables, a query table not built like `table`,
 * or null d_counts with n > 0. */
hg_status hg_intersect(const hg_table* table, const hg_table* queries,
                       uint32_t* d_counts, hipStream_t stream);

/* hg_count -- exact multiplicity of each query among the table's keys: the
 * query hashes to its bucket and every key of the bucket is compared
 * (Sec. 3.3 "Querying"; Sec. 5.4: the count of each key's appearances).
 *   d_queries  q keys of the table's key type; d_counts  q uint32 outputs.
 * Errors: HG_ERR_INVALID_ARG for a null table, or null pointers with q > 0,
 * or q >= 2^32. */
hg_status hg_count(const hg_table* table, const void* d_queries, uint64_t q,
                   uint32_t* d_counts, hipStream_t stream);

/* hg_query -- existence of each query: d_found[i] = 1 if the query occurs
 * among the keys, else 0 (Sec. 3.3 "Querying").  Same arguments and errors
 * as hg_count, with q uint8 outputs. */
hg_status hg_query(const hg_table* table, const void* d_queries, uint64_t q,
                   uint8_t* d_found, hipStream_t stream);

/* hg_count_ex / hg_query_ex -- hg_count / hg_query with an explicit probe
 * strategy (flags: 0 = library's choice, HG_PROBE_DIRECT, HG_PROBE_SORTED).
 * Results do not depend on the strategy.  Unknown flags: HG_ERR_INVALID_ARG. */
hg_status hg_count_ex(const hg_table* table, const void* d_queries, uint64_t q,
                      uint32_t* d_counts, uint32_t flags, hipStream_t stream);
hg_status hg_query_ex(const hg_table* table, const void* d_queries, uint64_t q,
                      uint8_t* d_found, uint32_t flags, hipStream_t stream);

/* hg_build_batched -- T independent tables in one call: table t holds keys
 * d_keys[o[t] .. o[t+1]) with o = d_table_offsets (device, T + 1 uint32,
 * o[0] = 0, non-decreasing, o[T] = n) and V_t = max(1, floor(n_t * num /
 * den)) buckets (opts->ratio_num / ratio_den; opts->P must be 1,
 * opts->num_buckets 0).  Each table is the HashGraph of Algorithm 1 over its
 * own keys; the batch is stored as one CSR over sum(V_t) buckets, in which
 * table t is "partition" t: hg_table_info reports P = T, part_offsets = o
 * and bucket_base[t] = first bucket of table t.  Offsets that break the
 * contract are clamped on the device to a non-decreasing sequence from 0 to
 * n (no fault; the tables then cover the clamped ranges).  Probe the result
 * with hg_count_batched / hg_query_batched only.  Errors: as hg_build, plus
 * HG_ERR_INVALID_ARG for T = 0, T > 2^22, null d_table_offsets, P != 1,
 * num_buckets != 0; HG_ERR_UNSUPPORTED for HG_BUILD_ATOMIC. */
hg_status hg_build_batched(const void* d_keys, uint64_t n, hg_key_type kt,
                           uint32_t num_tables, const uint32_t* d_table_offsets,
                           const hg_build_opts* opts, hipStream_t stream,
                           hg_table** out);

/* hg_count_batched / hg_query_batched -- probe a batched table: queries
 * d_queries[qo[t] .. qo[t+1]) go to table t (qo = d_query_offsets, device,
 * T + 1 uint32, same contract and clamping as the table offsets, qo[T] =
 * q).  Outputs as hg_count / hg_query, in query order.  Errors: as
 * hg_count, plus HG_ERR_INVALID_ARG for a table that is not batched or a
 * null d_query_offsets. */
hg_status hg_count_batched(const hg_table* table, const void* d_queries,
                           uint64_t q, const uint32_t* d_query_offsets,
                           uint32_t* d_counts, hipStream_t stream);
hg_status hg_query_batched(const hg_table* table, const void* d_queries,
                           uint64_t q, const uint32_t* d_query_offsets,
                           uint8_t* d_found, hipStream_t stream);

/* hg_bin_partition -- the hash-range split alone (Algorithm 2, Phase 2:
 * count per destination, prefix sum, scatter into a buffer), with P equal
 * hash ranges.  Writes d_out_keys[n] grouped by partition (order inside a
 * partition unspecified; Sec. 3.3 leaves it open) and d_part_offsets[P+1]
 * (part_offsets[P] = n).  The output is the send buffer of the exchange that
 * a multi-GPU build would run next.  d_out_keys must not overlap d_keys.
 * Errors: as hg_build for n and P; null outputs. */
hg_status hg_bin_partition(const void* d_keys, uint64_t n, hg_key_type kt,
                           uint32_t P, void* d_out_keys,
                           uint32_t* d_part_offsets, hipStream_t stream);

/* hg_bin_partition_noalloc -- hg_bin_partition for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, outputs and errors as
 * hg_bin_partition; it allocates nothing (no hipMalloc, hipFree or pool
 * call).  Its per-tile counts and scan sums live in a fixed scratch array of
 * 2^20 + 1024 words (4 MiB + 4 KiB) inside the library, one per device, kept
 * until the process ends: it holds P * ceil(n / 4096) <= 2^20 tile counts
 * and the scan's sums, i.e. n <= 2^28 keys for P = 16 or n <= 2^24 for
 * P = 256.  Larger requests return HG_ERR_INVALID_ARG (before anything is
 * enqueued).  Calls that
 * overlap on one device (other streams, other threads) share that array and
 * race: order them on one stream.  Every call rewrites all the scratch it
 * reads, so nothing has to be cleared between calls. */
hg_status hg_bin_partition_noalloc(const void* d_keys, uint64_t n,
                                   hg_key_type kt, uint32_t P,
                                   void* d_out_keys, uint32_t* d_part_offsets,
                                   hipStream_t stream);

/* hg_bin_partition_balanced -- the hash-range split with count-balanced
 * ranges (Algorithm 2, Phases 1 and 2; Sec. 3.3 "Phase 1: Multi-GPU Data
 * Partitioning"), P ranges for P devices.
 *   H(k) = hash(k) mod hash_range, 1 <= hash_range < 2^32 (the hash range
 *   HR of Sec. 3.3, e.g. the global table size).  The range is cut into
 *   bins of BinSize = ceil(HR / num_bins) consecutive values, bin =
 *   floor(H / BinSize), ceil(HR / BinSize) bins; num_bins 0 takes
 *   ceil(sqrt(HR)) (the paper's O(sqrt(HR))), num_bins <= 2^14.
 *   Boundary d (0 < d < P) is the first bin whose exclusive prefix count
 *   reaches floor(n * d / P) keys: d_bin_splits[0..P] (device, P+1 uint32;
 *   [0] = 0, [P] = number of bins, non-decreasing).  Partition d holds the
 *   keys with d_bin_splits[d] <= bin < d_bin_splits[d+1]; so the first d
 *   partitions hold between floor(n d / P) keys and that plus one bin's keys.
 *   d_out_keys[n]: the keys grouped by partition (order inside a partition
 *   unspecified); d_part_offsets[P+1] (device, part_offsets[P] = n).
 *   1 <= P <= 256 (any P, not only powers of two).  d_out_keys must not
 *   overlap d_keys.  Errors: HG_ERR_INVALID_ARG for P, hash_range or
 *   num_bins out of range, n >= 2^32, null outputs, or null keys with
 *   n > 0. */
hg_status hg_bin_partition_balanced(const void* d_keys, uint64_t n,
                                    hg_key_type kt, uint32_t P,
                                    uint64_t hash_range, uint32_t num_bins,
                                    void* d_out_keys, uint32_t* d_part_offsets,
                                    uint32_t* d_bin_splits, hipStream_t stream);

/* hg_hash_bucket -- the first loop of Algorithm 1 on its own: for each key,
 * d_hash[i] = hash(k) (uint64; for 32-bit keys the upper half is 0) and
 * d_bucket[i] = hash(k) mod V.  Either output may be null.  1 <= V < 2^32.
 * Exposed so the bucket map can be checked for any V without a table. */
hg_status hg_hash_bucket(const void* d_keys, uint64_t n, hg_key_type kt,
                         uint64_t V, uint64_t* d_hash, uint32_t* d_bucket,
                         hipStream_t stream);

/* hg_table_info -- fill *desc.  Reading num_buckets and probe_count_bytes
 * waits for the table's build to finish (both are computed on the device);
 * the other fields do not wait.  The device pointers stay owned by the
 * table. */
hg_status hg_table_info(const hg_table* table, hg_table_desc* desc);

/* hg_table_export -- copy the table's arrays into caller-owned device
 * buffers on `stream`: d_part_offsets[P+1], d_bucket_base[P+1],
 * d_offsets[num_buckets+1] and d_keys[n] (sizes from hg_table_info).  Any
 * destination may be null (skipped).  Errors: HG_ERR_INVALID_ARG for a null
 * table. */
hg_status hg_table_export(const hg_table* table, uint32_t* d_part_offsets,
                          uint32_t* d_bucket_base, uint32_t* d_offsets,
                          void* d_keys, hipStream_t stream);

/* hg_trim_pool -- hand cached device memory back to the system.  The
 * library allocates tables and workspace from a per-device cache of
 * hipMalloc blocks that keeps freed blocks for reuse: a freed block serves
 * the next request of its size on the same stream at once, and on other
 * streams once the work enqueued before its free has completed.  This
 * releases idle blocks of the current device, largest first, until at most
 * keep_bytes stay cached, waiting for each block's last use (callers that
 * share the device with other allocators, such as a serving loop, call it
 * after freeing tables).  The library also releases every idle block by
 * itself when hipMalloc fails, then tries once more.  Errors: HG_ERR_HIP. */
hg_status hg_trim_pool(uint64_t keep_bytes);

/* Device allocator hook (hg_set_allocator).
 *   alloc(bytes, stream, ctx) returns device memory of at least `bytes`
 *       bytes on the current device, aligned to 256 bytes and usable by work
 *       enqueued on `stream` from the moment of the call, or NULL when it
 *       cannot (the calling entry point then returns HG_ERR_OUT_OF_MEMORY).
 *   free_fn(ptr, bytes, stream, ctx) takes back a block in stream order: the
 *       stream's work enqueued before the call may still use it, so the
 *       block may only be handed to other streams after that work. */
typedef void* (*hg_alloc_fn)(size_t bytes, hipStream_t stream, void* ctx);
typedef void (*hg_free_fn)(void* ptr, size_t bytes, hipStream_t stream,
                           void* ctx);

/* hg_set_allocator -- route every device allocation of the library (table
 * memory and per-call workspace) through a caller-owned allocator, such as a
 * framework's caching allocator or an arena sized with hg_workspace_size,
 * instead of the library's block cache.  Both functions null restores the
 * cache.  The setting is process-wide and applies to calls that
 * start after it; a table remembers the allocator it was built with and
 * hg_table_free returns its memory there, so the allocator must outlive its
 * tables.  Errors: HG_ERR_INVALID_ARG when exactly one function is null.  A
 * block that is not 256-byte aligned fails the call that received it with
 * HG_ERR_INVALID_ARG (the block is handed back first). */
hg_status hg_set_allocator(hg_alloc_fn alloc, hg_free_fn free_fn, void* ctx);

/* Operations that hg_workspace_size can size. */
typedef enum hg_op {
  HG_OP_BUILD = 0,          /* hg_build(n keys of kt, opts)                */
  HG_OP_COUNT = 1,          /* hg_count_ex(table, n queries, flags = aux)  */
  HG_OP_QUERY = 2,          /* hg_query_ex(table, n queries, flags = aux)  */
  HG_OP_BUILD_BATCHED = 3,  /* hg_build_batched(n keys, aux tables, opts)  */
  HG_OP_COUNT_BATCHED = 4,  /* hg_count_batched(table, n queries)          */
  HG_OP_QUERY_BATCHED = 5,  /* hg_query_batched(table, n queries)          */
  HG_OP_BIN_PARTITION = 6   /* hg_bin_partition(n keys of kt, P = aux)     */
} hg_op;

/* hg_workspace_size -- the device memory that one call of `op` with these
 * arguments allocates, computed on the host without touching the device
 * (the sizes depend only on the arguments, never on key values).
 *   *workspace_bytes  temporary blocks, all live at once and handed back
 *                     before the call returns (in stream order),
 *   *table_bytes      blocks the new table keeps (builds only; else 0).
 * Each block is counted rounded up to a multiple of 256 bytes, so an arena
 * of workspace_bytes + table_bytes serves the call through hg_set_allocator
 * with any bump allocator that rounds the same way.  Arguments that the call
 * itself would reject give the same error here.  kt and opts are used by
 * the builds, table by the probes; aux holds the probe flags for COUNT and
 * QUERY, the number of tables for BUILD_BATCHED and P for BIN_PARTITION.  Either output may be
 * null.  Errors: HG_ERR_INVALID_ARG for an unknown op, and those of the
 * sized call. */
hg_status hg_workspace_size(hg_op op, const hg_table* table, uint64_t n,
                            hg_key_type kt, const hg_build_opts* opts,
                            uint32_t aux, uint64_t* workspace_bytes,
                            uint64_t* table_bytes);

/* hg_table_free -- release the table's memory in stream order on the stream
 * it was built on (to the allocator it was built with).  Work that uses the
 * table on other streams must be ordered before that stream's later work.
 * NULL is a no-op. */
void hg_table_free(hg_table* table);

/* Human-readable name of a status code (static storage). */
const char* hg_status_string(hg_status status);

/* Message of the last error on the calling thread ("" if none). */
const char* hg_last_error(void);

/* Per-kernel timing.  While enabled, every kernel launch of the library is
 * bracketed by HIP events on the stream it is launched on.
 * hg_profile_collect synchronizes those events, adds their durations to
 * per-kernel totals, and resets the event log; hg_profile_read copies up to
 * `cap` entries (name, launches, total milliseconds) and returns the number
 * of kernels seen.  hg_profile_reset clears the totals. */
hg_status hg_profile_enable(int on);
/* While `name` is not NULL, only launches of that name are bracketed (the
 * others run without events); NULL brackets every launch again.  The name
 * is copied.  A timing run can so keep the events of the one kernel it
 * reports and nothing else on the stream. */
hg_status hg_profile_only(const char* name);
hg_status hg_profile_collect(void);
int hg_profile_read(const char** names, uint64_t* launches, double* total_ms,
                    int cap);
void hg_profile_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* HG_H */
