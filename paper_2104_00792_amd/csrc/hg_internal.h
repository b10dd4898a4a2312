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

hipError_t launch_hist(int kt, const void* keys, uint32_t n, uint32_t log2P, uint32_t P,
                       const PartDesc* desc, uint32_t* cnt, hipStream_t s);
hipError_t launch_scatter(int kt, const void* keys, uint32_t n, uint32_t log2P, uint32_t P,
                          const PartDesc* desc, uint32_t* cursor, void* out, hipStream_t s);

hipError_t launch_probe(int kt, bool count, const void* tkeys, const uint32_t* offsets,
                        const PartDesc* desc, uint32_t log2P, uint32_t P, const void* queries,
                        uint32_t q, void* out, hipStream_t s);

hipError_t launch_hash_bucket(int kt, const void* keys, uint32_t n, uint32_t V, uint64_t* hash,
                              uint32_t* bucket, hipStream_t s);

}  // namespace hg
