// Launchers shared between the kernel translation unit and the C ABI layer.
// Every launcher enqueues one kernel on `s` and returns hipGetLastError().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hg_device.h"

namespace hg {

constexpr int kBlock = 256;                 // threads per workgroup
constexpr int kItems = 16;                  // keys per thread in a tile
constexpr int kTileKeys = kBlock * kItems;  // keys per tile
constexpr int kScanChunk = kBlock * 16;     // scan elements per workgroup
constexpr uint32_t kMaxP = 256;

inline uint32_t div_up(uint64_t a, uint64_t b) { return static_cast<uint32_t>((a + b - 1) / b); }

// ------------------------------------------------ the LDS-sorted path
// Keys (or queries) reach LDS-sized sub-bins of 2^log2S buckets through two
// stable multisplits: level 1 by partition or coarse bucket range (one
// segment, <= 256 digits, 4096-key tiles), level 2 by sub-bin inside each
// level-1 segment (<= kMaxD2 digits, kL2Threads x 16 (32-bit) or x 8 (64-bit)
// key tiles).  The LDS stages then sort (build) or probe one sub-bin per
// workgroup.
constexpr uint32_t kLog2SMax = 13;  // regular sub-bins: 2^log2S <= 2^13 buckets
constexpr uint32_t kLog2SMin = 10;
constexpr uint32_t kLog2SLds = 14;  // a segment's last sub-bin may grow to 2^14 in LDS
constexpr uint32_t kMaxD2 = 1024;
constexpr int kL1Threads = 256;
constexpr int kL1Items = 16;
constexpr int kL1Tile = kL1Threads * kL1Items;
constexpr int kL2Threads = 1024;      // level-2 scatter; counting takes half the threads, twice the items
constexpr int kLdsThreads = 1024;      // LDS probe workgroup
constexpr int kBuildThreads = 512;     // LDS build workgroup
constexpr uint32_t kMaxLog2W = 13;  // probe window: at most 2^13 buckets in LDS
constexpr uint32_t kProbeKeyCapBytes = 40 * 1024;  // table keys of one window in LDS

// Long buckets (more than kLongT keys) are left sorted by the build so that
// a probe counts them by binary search.  Buckets the build could not sort are
// listed in the table's `unsorted` block: word 0 holds their number, words
// 1 .. kMaxUnsorted their ids (when the number exceeds kMaxUnsorted, every
// long bucket is scanned).
constexpr uint32_t kLongT = 64;
constexpr uint32_t kMaxUnsorted = 256;
// The table's `unsorted` block also holds, after the ids, one word that the
// long-bucket pass sets to 1 when the table has any long bucket, else 0.
// Without long buckets no key occurs more than kLongT times, so a sorted
// probe carries its counts between kernels as bytes (launch_lds_probe,
// launch_tile_gather).
constexpr uint32_t kUnsortedWords = 2 + kMaxUnsorted;
constexpr uint32_t kHasLongWord = 1 + kMaxUnsorted;
static_assert(kLongT < 256, "a count of a table without long buckets fits a byte");
// Long buckets of at most kWaveLong keys are sorted by one wave each, longer
// ones by a workgroup.  Their ids share one list (the short ones from the
// front, the others from the back) of long_list_cap(n) entries, after
// kLongCtr counter words: [0] short ones, [2] long ones, [3] the work
// counter of the long ones, [4] the list's length, [5] the ones listed for
// a workgroup's register sort, placed right after the short ones ([1],
// [6..7] unused).  A bucket appears at most once in each of the three, so
// three entries per possible long bucket always suffice.
constexpr uint32_t kWaveLong = 4096;
constexpr uint32_t kLongCtr = 8;
inline uint64_t long_list_cap(uint64_t n) { return 3 * (n / (kLongT + 1) + 1); }
constexpr int kLongThreads = 1024;
constexpr uint32_t kLongGrid = 512;  // resident workgroups (two per CU)

// Long buckets of an atomic-path build: appended to long_list.
hipError_t launch_find_long(const uint32_t* offsets, const uint32_t* num_buckets_dev, uint64_t bound,
                            uint32_t* long_count, uint32_t* long_list, hipStream_t s);
// Long buckets of more than kBigChunk keys are shared by many workgroups,
// one chunk of kBigChunk keys each: chunk sets of distinct keys, one merge
// per bucket, then the rewrite chunk by chunk.  Their bookkeeping lives in a
// workspace of big_words(n, key bytes) u32 words.
constexpr uint32_t kBigChunk = 1u << 16;
constexpr uint32_t kSetMax = 64;  // distinct keys a long bucket may have to be rewritten as runs
constexpr uint32_t kOver = 0xFFFFFFFFu;  // marks more than kSetMax distinct keys
inline uint64_t big_buckets_max(uint64_t n) { return n / kBigChunk + 1; }
inline uint64_t big_words(uint64_t n, uint32_t ks) {
  const uint64_t nb = big_buckets_max(n), nc = 2 * nb;
  return 4 + 2 * nb + 3 * nc + nc * kSetMax * (1 + ks / 4) + nb * (1 + (kSetMax + 1) + kSetMax * ks / 4) + 4;
}

// Sort every listed long bucket in place (persistent workgroups; long_ctr
// and long_list as above; `big` a workspace of big_words(n, ks) words for n
// keys).
hipError_t launch_long_sort(int kt, const uint32_t* offsets, uint32_t* long_ctr, uint32_t* long_list, void* keys,
                            uint32_t* unsorted, uint32_t* big, uint64_t n, hipStream_t s);

inline int l2_tile_keys(int kt) { return kL2Threads * (kt == 0 ? 8 : 4); }
// Level-2 tiles of a segment start at its first key rounded down to this
// many keys: interior tiles take vector loads, and every tile's keys, slots
// (u16) and counts start on a 128-byte line, so that no wave's access
// straddles one more line than it fills.
constexpr uint32_t kTileAlign = 64;

// Segments of the level-2 split and sub-bins of the LDS stages, computed on
// the device (no host round trip).  Segment s holds keys key0[s] .. key0[s+1]
// of the level-1 output and global buckets g0[s] .. g0[s+1]; it has T[s]
// level-2 tiles and D[s] sub-bins; its per-tile digit counts start at
// cbase[s] and are laid out [digit][tile].  tile_seg[b] / sb_seg[b] name
// the segment of level-2 tile b / sub-bin b.  The arrays live in device
// memory after the header, which the plan kernels fill in.  desc_by_seg: the
// segments are separate tables (batched build) and segment s maps hashes to
// buckets with descriptor s; otherwise a key's descriptor is its hash
// partition's.
struct SegPlan {
  uint32_t nseg, total_tiles, total_counts, total_subbins;
  uint32_t num_buckets, n, tile_keys, log2S;
  uint32_t desc_by_seg, max_tiles, max_subbins, pad;
  uint32_t* key0;
  uint32_t* g0;
  uint32_t* D;
  uint32_t* T;
  uint32_t* tile_first;
  uint32_t* cbase;
  uint32_t* sb_first;
  uint32_t* tile_seg;
  uint32_t* sb_seg;
};
constexpr uint32_t kPlanArrays = 7;
constexpr uint32_t kMaxTables = 1u << 22;  // batched tables per call

// Bytes of a plan with room for max_seg segments, max_tiles level-2 tiles
// and max_subbins sub-bins.
inline size_t plan_bytes(uint32_t max_seg, uint32_t max_tiles, uint32_t max_subbins) {
  return (sizeof(SegPlan) + 255) / 256 * 256 +
         sizeof(uint32_t) * (kPlanArrays * (static_cast<size_t>(max_seg) + 1) + max_tiles + max_subbins);
}

// DIG_RANGE (level 1 only): desc[0] maps a key to H = hash mod HR, and the
// P + 1 u32 right after desc[0] are range starts (bounds[0] = 0,
// non-decreasing); the digit is the last d < nd with bounds[d] <= H.
enum DigitKind { DIG_PART = 0, DIG_COARSE = 1, DIG_SUB = 2, DIG_RANGE = 3 };
enum SplitOp { OP_COUNT = 0, OP_SCATTER = 1 };

// One split pass.  level 1: a single segment [0, n) with nd <= 256 digits and
// grid ceil(n / kL1Tile); level 2: segments from `plan` (<= kMaxD2 digits
// each), grid max_tiles.  dig/shift: DIG_PART (partition), DIG_COARSE (global
// bucket >> shift, capped at nd - 1), DIG_SUB (bucket offset in the segment
// >> shift, capped).  COUNT writes per-tile digit counts; SCATTER moves `in`
// to `out` using the scanned counts and, when perm is not null, writes
// perm[i] = slot of in[i] among its tile's keys in digit order.
hipError_t launch_msplit(int kt, int level, int op, int dig, const void* in, uint32_t n, uint32_t max_tiles,
                         const SegPlan* plan, uint32_t nd, uint32_t log2P, uint32_t P, const PartDesc* desc,
                         uint32_t shift, uint32_t* counts, void* out, uint16_t* perm, hipStream_t s);

// Inverse of a split (same level, tiles, plan and scanned counts) applied to
// u32 values: out[i] = src[position of key i after the split], or that value
// != 0 as bytes.  perm as written by the split's SCATTER.
// out_kind: GATHER_STAGE writes the values in the width they came in (bytes
// when the table has no long bucket, see kHasLongWord; else u32), for a
// further gather; GATHER_COUNT writes u32 counts, GATHER_FOUND bytes 0/1.
// `unsorted` is the table's block that holds the long-bucket word.
enum GatherOut { GATHER_STAGE = 0, GATHER_COUNT = 1, GATHER_FOUND = 2 };
hipError_t launch_tile_gather(int kt, int level, const uint16_t* perm, const void* src, uint32_t n,
                              uint32_t max_tiles, const SegPlan* plan, uint32_t nd, const uint32_t* scan,
                              const uint32_t* unsorted, void* out, int out_kind, hipStream_t s);

// Count-balanced ranges (Algorithm 2, Phase 1): kMaxBins bins at most.
constexpr uint32_t kMaxBins = 1u << 14;
// counts[b] += keys with floor((hash mod HR) / bin_size) == b, b < nbins
// (counts zeroed by the caller).
hipError_t launch_bin_hist(int kt, const void* keys, uint32_t n, uint32_t HR, uint32_t bin_size, uint32_t nbins,
                           uint32_t* counts, hipStream_t s);
// From the scanned bin counts: splits[0..P] (first bin whose prefix reaches
// floor(n d / P); splits[0] = 0, splits[P] = nbins) and the DIG_RANGE
// descriptor at rdesc (mod HR, then bounds[d] = min(splits[d] * bin_size, HR)).
hipError_t launch_range_splits(const uint32_t* bin_offset, uint32_t nbins, uint32_t n, uint32_t P, uint32_t HR,
                               uint32_t bin_size, uint32_t* splits, PartDesc* rdesc, hipStream_t s);

// Plan of the level-2 split, written into `plan` (plan_bytes(nseg,
// max_tiles, max_subbins) bytes; the level-2 grid is max_tiles, the sub-bin
// grid max_subbins).
// mode 0: segments are the level-1 partition digits (key0 from the scanned
// level-1 counts scan1 [digit][tile], g0 = bucket_base); mode 1: coarse
// bucket ranges of 2^sh1; mode 2: batched tables (key0 = seg_keys, g0 =
// bucket_base, one descriptor per segment).  *nb_total is the number of
// buckets.  Writes offsets[num_buckets] = n when offsets is not null.
hipError_t launch_plan(const uint32_t* scan1, uint32_t tiles1, uint32_t nseg, uint32_t n, int mode,
                       const uint32_t* bucket_base, const uint32_t* nb_total, const uint32_t* seg_keys, uint32_t sh1,
                       uint32_t log2S, uint32_t tile2, uint32_t max_tiles, uint32_t max_subbins, uint32_t* offsets,
                       SegPlan* plan, hipStream_t s);

// Table layout of a batch of T tables with keys table_keys[t] ..
// table_keys[t+1] (n keys in all): part_offsets[0..T] = the offsets clamped
// to a non-decreasing sequence from 0 to n; with bucket_base not null also
// V_t = max(1, floor(n_t * num / den)), bucket_base[0..T] and desc[0..T).
// One workgroup.
hipError_t launch_batch_layout(const uint32_t* table_keys, uint32_t T, uint32_t n, uint32_t num, uint32_t den,
                               uint32_t* part_offsets, uint32_t* bucket_base, PartDesc* desc, hipStream_t s);

// One workgroup per sub-bin: LDS counting sort of its keys by bucket; writes
// the sub-bin's CSR offsets and keys.  grid = max_subbins.
// Sub-bins of more than 65535 keys are shared by several workgroups
// (heavy passes); their workspace `heavy` holds 2 + 2 * max_chunks +
// max_heavy words, max_chunks = n / heavy_chunk_keys() + max_heavy + 1 and
// max_heavy = n / 65536 + 1.  `long_flags` (max_subbins words) marks the
// 32-bit sub-bins whose long buckets a later pass lists.
uint32_t heavy_chunk_keys();
hipError_t launch_lds_build(int kt, const void* in, const SegPlan* plan, const uint32_t* scan2, uint32_t max_subbins,
                            uint32_t log2P, uint32_t P, const PartDesc* desc, uint32_t* offsets, void* out,
                            uint32_t* long_count, uint32_t* long_list, uint32_t* heavy, uint32_t max_chunks,
                            uint32_t* long_flags, hipStream_t s);

// Queries of one sub-bin, at most probe_chunk_keys() per workgroup (a
// sub-bin with more is shared through a queue): windows of 2^log2W buckets
// of the table (offsets and keys) in LDS; counts in the split order, as
// bytes when the table has no long bucket (kHasLongWord), else as u32.
// Workspace: queue[1 + 2 * (q / probe_chunk_keys(kt) + 1)] (a small kernel
// lists the chunks of every sub-bin with more queries first).  A workgroup
// holds kProbeReg(kt) queries per thread (fewer 64-bit ones, so that the
// kernel keeps within 64 VGPRs and two workgroups share a CU).
constexpr int kProbeReg32 = 20;
constexpr int kProbeReg64 = 10;
uint32_t probe_chunk_keys(int kt);
hipError_t launch_lds_probe(int kt, const void* q2, const SegPlan* qplan, const uint32_t* qscan2,
                            uint32_t max_subbins, uint32_t q, uint32_t log2P, uint32_t P, const PartDesc* desc,
                            const uint32_t* offsets, const void* tkeys, const uint32_t* unsorted, uint32_t log2W,
                            uint32_t* queue, void* c2, hipStream_t s);

// kt: 0 = 32-bit keys, 1 = 64-bit keys.
hipError_t launch_fill_u32(uint32_t* p, uint64_t len, uint32_t value, hipStream_t s);

hipError_t launch_part_count(int kt, const void* keys, uint32_t n, uint32_t log2P,
                             uint32_t num_tiles, uint32_t* tile_counts, hipStream_t s);
hipError_t launch_part_scatter(int kt, const void* keys, uint32_t n, uint32_t log2P,
                               uint32_t num_tiles, const uint32_t* tile_base, void* out,
                               hipStream_t s);

// Exclusive scan in place of a[0 .. len), len = *len_dev if len_dev is not
// null (then len_bound bounds it), else len_bound.  block_sums holds
// div_up(len_bound, kScanChunk) words.
hipError_t launch_scan_exclusive(uint32_t* a, const uint32_t* len_dev, uint64_t len_bound,
                                 uint32_t* block_sums, hipStream_t s);

// Partition offsets, table sizes, bucket bases and bucket-map descriptors.
// tile_base may be null when P == 1.  bucket_base / desc may be null
// (partition offsets only).
hipError_t launch_layout(const uint32_t* tile_base, uint32_t num_tiles, uint32_t P, uint32_t n,
                         uint32_t num, uint32_t den, uint64_t V_plain, uint32_t* part_offsets,
                         uint32_t* bucket_base, PartDesc* desc, hipStream_t s);

// As launch_layout, with the table sizes and bucket bases copied from the
// descriptors `src` of another table (P of them).
hipError_t launch_layout_like(const uint32_t* tile_base, uint32_t num_tiles, uint32_t P, uint32_t n,
                              const PartDesc* src, uint32_t* part_offsets, uint32_t* bucket_base, PartDesc* desc,
                              hipStream_t s);

hipError_t launch_hist(int kt, const void* keys, uint32_t n, uint32_t log2P, uint32_t P,
                       const PartDesc* desc, uint32_t* cnt, hipStream_t s);
hipError_t launch_scatter(int kt, const void* keys, uint32_t n, uint32_t log2P, uint32_t P,
                          const PartDesc* desc, uint32_t* cursor, void* out, hipStream_t s);

hipError_t launch_probe(int kt, bool count, const void* tkeys, const uint32_t* offsets,
                        const PartDesc* desc, uint32_t log2P, uint32_t P, const uint32_t* unsorted,
                        const void* queries, uint32_t q, void* out, hipStream_t s);

hipError_t launch_hash_bucket(int kt, const void* keys, uint32_t n, uint32_t V, uint64_t* hash,
                              uint32_t* bucket, hipStream_t s);

}  // namespace hg
