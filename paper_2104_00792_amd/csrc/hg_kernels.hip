// HashGraph kernels for gfx950 (wave64, 160 KiB LDS per CU).
//
// Build (Algorithm 1 of Tripathy & Green, arXiv 2104.00792): hash + bucket,
// histogram of bucket sizes, exclusive prefix sum into the CSR offsets,
// scatter of the keys.  With P > 1 the keys are first split into hash-range
// partitions (Algorithm 2, Phase 2): per-tile partition counts, a prefix sum
// over (partition, tile), and a stable scatter.  Probe: hash the query, read
// its bucket's offset range, compare every key of the bucket (Sec. 3.3
// "Querying"; exact counts as in Sec. 5.4).
//
// Every kernel reads keys in 16-byte vector loads when a tile is whole and the
// base is 16-byte aligned, and recomputes the hash instead of storing it
// (the paper materialises H_A; recomputing saves 8 bytes per key per pass).
#include "hg_internal.h"
#include "hg_tile.h"

namespace hg {
namespace {

constexpr int kWaves = kBlock / kWave;

template <typename K> struct Vec {
  static constexpr int kPer = 16 / sizeof(K);   // keys per 16-byte load
  static constexpr int kLoads = kItems / kPer;  // loads per thread per tile
};

// Position inside its tile of item i (load i / kPer, component i % kPer) of
// thread t: each 16-byte load of a wave covers 64 * 16 contiguous bytes.
template <typename K>
__device__ __forceinline__ uint32_t tile_index(int i, uint32_t t) {
  constexpr int P = Vec<K>::kPer;
  return (static_cast<uint32_t>(i / P) * kBlock + t) * P + static_cast<uint32_t>(i % P);
}

// Loads tile `tile` of src[0, n) into v; bit i of the result marks item i as
// inside the array.
template <typename K>
__device__ __forceinline__ uint32_t load_tile(const K* __restrict__ src, uint32_t n, uint32_t tile,
                                              K (&v)[kItems]) {
  const uint64_t start = static_cast<uint64_t>(tile) * kTileKeys;
  const uint32_t t = threadIdx.x;
  constexpr int P = Vec<K>::kPer;
  if (start + kTileKeys <= n && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
    const uint4* p = reinterpret_cast<const uint4*>(src + start);
#pragma unroll
    for (int j = 0; j < Vec<K>::kLoads; ++j) {
      const uint4 x = p[j * kBlock + t];
      K tmp[P];
      __builtin_memcpy(tmp, &x, 16);
#pragma unroll
      for (int c = 0; c < P; ++c) v[j * P + c] = tmp[c];
    }
    return (1u << kItems) - 1u;
  }
  uint32_t mask = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint64_t e = start + tile_index<K>(i, t);
    if (e < n) {
      v[i] = src[e];
      mask |= 1u << i;
    } else {
      v[i] = 0;
    }
  }
  return mask;
}

// ------------------------------------------------------------------ fill
__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* __restrict__ p, uint64_t len, uint32_t value) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kBlock;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < len; i += stride) p[i] = value;
}

// ------------------------------------------------------------- scans (a3, a6)
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ a, const uint32_t* len_dev,
                                                        uint64_t len_bound, uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t wtot[kWaves];
  const uint64_t len = len_dev ? static_cast<uint64_t>(*len_dev) : len_bound;
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanChunk;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanChunk / kBlock; ++j) {
    const uint64_t e = base + static_cast<uint64_t>(j) * kBlock + threadIdx.x;
    if (e < len) s += a[e];
  }
  uint32_t total;
  block_exclusive_sum<kBlock>(s, wtot, total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_spine(uint32_t* __restrict__ bs, uint32_t nb) {
  __shared__ uint32_t wtot[kWaves];
  constexpr int kPer = 16;
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < nb; c0 += kBlock * kPer) {
    uint32_t x[kPer];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const uint32_t idx = c0 + threadIdx.x * kPer + j;
      x[j] = idx < nb ? bs[idx] : 0u;
      s += x[j];
    }
    uint32_t total;
    uint32_t run = carry + block_exclusive_sum<kBlock>(s, wtot, total);
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const uint32_t idx = c0 + threadIdx.x * kPer + j;
      if (idx < nb) bs[idx] = run;
      run += x[j];
    }
    carry += total;
  }
}

// kPrefix: the chunk's prefix is the sum of block_sums[0 .. blockIdx.x),
// added up here by the whole workgroup (the block sums are not scanned
// first); otherwise block_sums holds the scanned prefixes.
template <bool kPrefix>
__global__ __launch_bounds__(kBlock) void k_scan_down(uint32_t* __restrict__ a, const uint32_t* len_dev,
                                                      uint64_t len_bound, const uint32_t* __restrict__ block_sums) {
  constexpr int kPer = kScanChunk / kBlock;  // 16
  __shared__ uint32_t buf[kScanChunk + kScanChunk / kPer];
  __shared__ uint32_t wtot[kWaves];
  const uint64_t len = len_dev ? static_cast<uint64_t>(*len_dev) : len_bound;
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanChunk;
  if (base >= len) return;  // whole workgroup leaves together
  const uint32_t t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const uint32_t i = j * kBlock + t;
    const uint64_t e = base + i;
    buf[i + i / kPer] = e < len ? a[e] : 0u;
  }
  uint32_t prefix = 0;
  if (kPrefix) {
    uint32_t part = 0;
    for (uint32_t i = t; i < blockIdx.x; i += kBlock) part += block_sums[i];
    block_exclusive_sum<kBlock>(part, wtot, prefix);
  } else {
    prefix = block_sums[blockIdx.x];
  }
  __syncthreads();
  uint32_t x[kPer];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const uint32_t i = t * kPer + j;
    x[j] = buf[i + i / kPer];
    s += x[j];
  }
  uint32_t total;
  uint32_t run = prefix + block_exclusive_sum<kBlock>(s, wtot, total);
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const uint32_t i = t * kPer + j;
    buf[i + i / kPer] = run;
    run += x[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const uint32_t i = j * kBlock + t;
    const uint64_t e = base + i;
    if (e < len) a[e] = buf[i + i / kPer];
  }
}

// ----------------------------------------------------------------- layout
// Partition offsets from the scanned tile counts; table sizes
// V_p = max(1, floor(n_p * num / den)) (or V_plain); bucket bases; the
// bucket-map reciprocals.  One workgroup; P <= 256.
__global__ __launch_bounds__(kBlock) void k_layout(const uint32_t* __restrict__ tile_base, uint32_t num_tiles,
                                                   uint32_t P, uint32_t n, uint32_t num, uint32_t den,
                                                   uint64_t V_plain, uint32_t* __restrict__ po,
                                                   uint32_t* __restrict__ bb, PartDesc* __restrict__ desc) {
  __shared__ uint32_t spo[kMaxP + 1];
  __shared__ uint32_t wtot[kWaves];
  const uint32_t t = threadIdx.x;
  if (t < P) spo[t] = (tile_base != nullptr && num_tiles != 0) ? tile_base[static_cast<uint64_t>(t) * num_tiles] : 0u;
  if (t == 0) spo[P] = n;
  __syncthreads();
  if (t < P) po[t] = spo[t];
  if (t == 0) po[P] = n;
  if (bb == nullptr) return;  // uniform over the workgroup
  uint32_t V = 0;
  if (t < P) {
    const uint64_t np = spo[t + 1] - spo[t];
    uint64_t v = (P == 1 && V_plain != 0) ? V_plain : np * num / den;
    if (v < 1) v = 1;
    V = static_cast<uint32_t>(v);
  }
  uint32_t total;
  const uint32_t ex = block_exclusive_sum<kBlock>(V, wtot, total);
  if (t < P) {
    desc[t] = make_desc(V, ex);
    bb[t] = ex;
  }
  if (t == 0) bb[P] = total;
}

// Layout of a table built like another (the query table of Sec. 3.3): the
// partition offsets from the scanned tile counts, every table size and
// bucket base copied from the source table, so that bucket g of both tables
// holds the keys that hash to g.  One workgroup; P <= 256.
__global__ __launch_bounds__(kBlock) void k_layout_like(const uint32_t* __restrict__ tile_base, uint32_t num_tiles,
                                                        uint32_t P, uint32_t n, const PartDesc* __restrict__ src,
                                                        uint32_t* __restrict__ po, uint32_t* __restrict__ bb,
                                                        PartDesc* __restrict__ desc) {
  const uint32_t t = threadIdx.x;
  if (t < P) {
    po[t] = (tile_base != nullptr && num_tiles != 0) ? tile_base[static_cast<uint64_t>(t) * num_tiles] : 0u;
    const PartDesc d = src[t];
    desc[t] = d;
    bb[t] = d.base;
  }
  if (t == 0) {
    po[P] = n;
    bb[P] = src[P - 1].base + src[P - 1].V;
  }
}

// ------------------------------------- count-balanced ranges (Alg. 2, Phase 1)
// Keys per bin of the reduced hash range: H = hash(k) mod HR, bin =
// floor(H / bin_size).  A persistent grid; a workgroup counts its share in
// LDS (eight keys per thread in flight), then adds its nonzero counters to
// the global ones.
constexpr int kBinThreads = 1024;
constexpr int kBinItems = 8;

template <typename K>
__global__ __launch_bounds__(kBinThreads) void k_bin_hist(const K* __restrict__ keys, uint32_t n, uint32_t HR,
                                                          uint32_t bin_size, uint32_t nbins,
                                                          uint32_t* __restrict__ counts) {
  __shared__ uint32_t hist[kMaxBins];
  const uint32_t t = threadIdx.x;
  for (uint32_t i = t; i < nbins; i += kBinThreads) hist[i] = 0;
  const uint32_t m_hr = recip32(HR), m_bs = recip32(bin_size);
  const uint64_t m_hr64 = recip64(HR);
  __syncthreads();
  constexpr uint64_t kStep = kBinThreads * kBinItems;
  // 64-bit positions: n may come within one step of 2^32.
  for (uint64_t base = blockIdx.x * kStep; base < n; base += gridDim.x * kStep) {
    K v[kBinItems];
#pragma unroll
    for (int u = 0; u < kBinItems; ++u) {
      const uint64_t i = base + static_cast<uint64_t>(u) * kBinThreads + t;
      v[u] = keys[i < n ? i : n - 1];
    }
#pragma unroll
    for (int u = 0; u < kBinItems; ++u) {
      const uint32_t H = mod_by_recip(KeyTraits<K>::hash(v[u]), HR, m_hr, m_hr64);
      const uint32_t b = quot_by_recip(H, bin_size, m_bs);
      if (base + static_cast<uint64_t>(u) * kBinThreads + t < n) atomicAdd(&hist[b], 1u);
    }
  }
  __syncthreads();
  for (uint32_t i = t; i < nbins; i += kBinThreads)
    if (hist[i] != 0) atomicAdd(&counts[i], hist[i]);
}

// One workgroup: the range boundaries from the scanned bin counts (entry
// nbins of the prefix sums is n), and the DIG_RANGE descriptor.
__global__ __launch_bounds__(kBlock) void k_range_splits(const uint32_t* __restrict__ bin_offset, uint32_t nbins,
                                                         uint32_t n, uint32_t P, uint32_t HR, uint32_t bin_size,
                                                         uint32_t* __restrict__ splits,
                                                         PartDesc* __restrict__ rdesc) {
  uint32_t* bounds = reinterpret_cast<uint32_t*>(rdesc + 1);
  for (uint32_t d = threadIdx.x; d <= P; d += kBlock) {
    uint32_t sp = d == 0 ? 0u : nbins;
    if (d > 0 && d < P) {
      const uint64_t target = static_cast<uint64_t>(n) * d / P;
      uint32_t lo = 0, hi = nbins + 1;  // first x in [0, nbins] with prefix(x) >= target
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        const uint32_t v = mid == nbins ? n : bin_offset[mid];
        if (v < target)
          lo = mid + 1;
        else
          hi = mid;
      }
      sp = lo;
    }
    splits[d] = sp;
    const uint64_t hb = static_cast<uint64_t>(sp) * bin_size;
    bounds[d] = static_cast<uint32_t>(hb < HR ? hb : HR);
  }
  if (threadIdx.x == 0) {
    rdesc[0] = make_desc(HR, 0);
  }
}

// ------------------------------------------------ histogram and scatter (a5, a7)
// One atomic per lane, except that the lanes sharing the first active lane's
// bucket are combined into a single atomic (duplicate-heavy inputs).
template <bool kReturn>
__device__ __forceinline__ uint32_t aggregated_add(uint32_t* __restrict__ ctr, uint32_t g, bool valid) {
  const uint64_t act = ballot(valid);
  if (act == 0) return 0;
  const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<long long>(act)) - 1);
  const uint32_t gl = readlane(g, leader);
  const bool in = valid && g == gl;
  const uint64_t same = ballot(in);
  uint32_t base = 0;
  if (lane_id() == leader) {
    if (kReturn)
      base = atomicAdd(&ctr[gl], popc64(same));
    else
      atomicAdd(&ctr[gl], popc64(same));
  }
  uint32_t pos = 0;
  if (kReturn) {
    base = readlane(base, leader);
    if (in) pos = base + popc64(same & lanemask_lt());
    else if (valid) pos = atomicAdd(&ctr[g], 1u);
  } else if (valid && !in) {
    atomicAdd(&ctr[g], 1u);
  }
  return pos;
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_hist(const K* __restrict__ keys, uint32_t n, uint32_t log2P, uint32_t P,
                                                 const PartDesc* __restrict__ desc, uint32_t* __restrict__ cnt) {
  __shared__ PartDesc sd[kMaxP];
  for (uint32_t i = threadIdx.x; i < P; i += kBlock) sd[i] = desc[i];
  __syncthreads();
  K v[kItems];
  const uint32_t mask = load_tile(keys, n, blockIdx.x, v);
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const bool valid = (mask >> i) & 1u;
    uint32_t g = 0;
    if (valid) {
      const auto h = KeyTraits<K>::hash(v[i]);
      g = global_bucket(h, sd[part_of(h, log2P)]);
    }
    aggregated_add<false>(cnt, g, valid);
  }
}

// cursor[g] starts at the first position of bucket g and ends at the first
// position of bucket g + 1 (the CSR offsets shifted by one).
template <typename K>
__global__ __launch_bounds__(kBlock) void k_scatter(const K* __restrict__ keys, uint32_t n, uint32_t log2P, uint32_t P,
                                                    const PartDesc* __restrict__ desc, uint32_t* __restrict__ cursor,
                                                    K* __restrict__ out) {
  __shared__ PartDesc sd[kMaxP];
  for (uint32_t i = threadIdx.x; i < P; i += kBlock) sd[i] = desc[i];
  __syncthreads();
  K v[kItems];
  const uint32_t mask = load_tile(keys, n, blockIdx.x, v);
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const bool valid = (mask >> i) & 1u;
    uint32_t g = 0;
    if (valid) {
      const auto h = KeyTraits<K>::hash(v[i]);
      g = global_bucket(h, sd[part_of(h, log2P)]);
    }
    const uint32_t pos = aggregated_add<true>(cursor, g, valid);
    if (valid) out[pos] = v[i];
  }
}

// ------------------------------------------------------------- probe (a8)
template <typename K, bool kCount>
__global__ __launch_bounds__(kBlock) void k_probe(const K* __restrict__ tkeys, const uint32_t* __restrict__ offs,
                                                  const PartDesc* __restrict__ desc, uint32_t log2P, uint32_t P,
                                                  const uint32_t* __restrict__ unsorted, const K* __restrict__ qs,
                                                  uint32_t q, void* __restrict__ out) {
  __shared__ PartDesc sd[kMaxP];
  for (uint32_t i = threadIdx.x; i < P; i += kBlock) sd[i] = desc[i];
  __syncthreads();
  K v[kItems];
  const uint32_t mask = load_tile(qs, q, blockIdx.x, v);
  uint32_t lo[kItems], hi[kItems], gb[kItems];
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    gb[i] = 0;
    if ((mask >> i) & 1u) {
      const auto h = KeyTraits<K>::hash(v[i]);
      gb[i] = global_bucket(h, sd[part_of(h, log2P)]);
      lo[i] = offs[gb[i]];
      hi[i] = offs[gb[i] + 1];
    } else {
      lo[i] = hi[i] = 0;
    }
  }
  const uint32_t nuns = unsorted[0];
  const uint64_t start = static_cast<uint64_t>(blockIdx.x) * kTileKeys;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if ((mask >> i) & 1u) {
      const bool srt = hi[i] - lo[i] > kLongT && long_bucket_sorted(unsorted, nuns, gb[i], kMaxUnsorted);
      const uint32_t c = count_equal(tkeys, lo[i], hi[i], v[i], srt);
      const uint64_t e = start + tile_index<K>(i, threadIdx.x);
      if (kCount)
        static_cast<uint32_t*>(out)[e] = c;
      else
        static_cast<uint8_t*>(out)[e] = c != 0 ? 1 : 0;
    }
  }
}

// --------------------------------------------------------- hash + bucket (a1)
template <typename K>
__global__ __launch_bounds__(kBlock) void k_hash_bucket(const K* __restrict__ keys, uint32_t n, PartDesc d,
                                                        uint64_t* __restrict__ hash, uint32_t* __restrict__ bucket) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kBlock;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
    const auto h = KeyTraits<K>::hash(keys[i]);
    if (hash) hash[i] = static_cast<uint64_t>(h);
    if (bucket) bucket[i] = global_bucket(h, d);  // the tables' own map (base 0)
  }
}

inline uint32_t grid_for(uint64_t len) {
  const uint64_t b = (len + kBlock - 1) / kBlock;
  return static_cast<uint32_t>(b < 8192 ? (b == 0 ? 1 : b) : 8192);
}

}  // namespace

// ================================================================ launchers
hipError_t launch_fill_u32(uint32_t* p, uint64_t len, uint32_t value, hipStream_t s) {
  if (len == 0) return hipSuccess;
  k_fill_u32<<<grid_for(len), kBlock, 0, s>>>(p, len, value);
  return hipGetLastError();
}

// The partition split is the level-1 multisplit with partition digits
// (4096-key tiles, counts laid out [partition][tile]).
hipError_t launch_part_count(int kt, const void* keys, uint32_t n, uint32_t log2P, uint32_t num_tiles,
                             uint32_t* tile_counts, hipStream_t s) {
  (void)num_tiles;
  return launch_msplit(kt, 1, OP_COUNT, DIG_PART, keys, n, 0, nullptr, 1u << log2P, log2P, 1u << log2P, nullptr, 0,
                       tile_counts, nullptr, nullptr, s);
}

hipError_t launch_part_scatter(int kt, const void* keys, uint32_t n, uint32_t log2P, uint32_t num_tiles,
                               const uint32_t* tile_base, void* out, hipStream_t s) {
  (void)num_tiles;
  return launch_msplit(kt, 1, OP_SCATTER, DIG_PART, keys, n, 0, nullptr, 1u << log2P, log2P, 1u << log2P, nullptr, 0,
                       const_cast<uint32_t*>(tile_base), out, nullptr, s);
}

hipError_t launch_scan_exclusive(uint32_t* a, const uint32_t* len_dev, uint64_t len_bound, uint32_t* block_sums,
                                 hipStream_t s) {
  if (len_bound == 0) return hipSuccess;
  const uint32_t nb = div_up(len_bound, kScanChunk);
  k_scan_reduce<<<nb, kBlock, 0, s>>>(a, len_dev, len_bound, block_sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Up to kScanFusedBlocks chunks, each down-sweep workgroup adds up the
  // sums before its chunk itself (at most that many loads, from L2): one
  // launch and one single-workgroup kernel fewer.  Longer scans scan the
  // block sums first.
  constexpr uint32_t kScanFusedBlocks = 4096;
  if (nb <= kScanFusedBlocks) {
    k_scan_down<true><<<nb, kBlock, 0, s>>>(a, len_dev, len_bound, block_sums);
    return hipGetLastError();
  }
  k_scan_spine<<<1, kBlock, 0, s>>>(block_sums, nb);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scan_down<false><<<nb, kBlock, 0, s>>>(a, len_dev, len_bound, block_sums);
  return hipGetLastError();
}

hipError_t launch_layout_like(const uint32_t* tile_base, uint32_t num_tiles, uint32_t P, uint32_t n,
                              const PartDesc* src, uint32_t* part_offsets, uint32_t* bucket_base, PartDesc* desc,
                              hipStream_t s) {
  k_layout_like<<<1, kBlock, 0, s>>>(tile_base, num_tiles, P, n, src, part_offsets, bucket_base, desc);
  return hipGetLastError();
}

hipError_t launch_bin_hist(int kt, const void* keys, uint32_t n, uint32_t HR, uint32_t bin_size, uint32_t nbins,
                           uint32_t* counts, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (nbins == 0 || nbins > kMaxBins || HR == 0 || bin_size == 0) return hipErrorInvalidValue;
  constexpr uint32_t kStep = kBinThreads * kBinItems;
  const uint32_t chunks = div_up(n, kStep);
  const uint32_t grid = chunks < 512u ? chunks : 512u;
  if (kt == 0)
    k_bin_hist<uint32_t><<<grid, kBinThreads, 0, s>>>(static_cast<const uint32_t*>(keys), n, HR, bin_size, nbins,
                                                      counts);
  else
    k_bin_hist<uint64_t><<<grid, kBinThreads, 0, s>>>(static_cast<const uint64_t*>(keys), n, HR, bin_size, nbins,
                                                      counts);
  return hipGetLastError();
}

hipError_t launch_range_splits(const uint32_t* bin_offset, uint32_t nbins, uint32_t n, uint32_t P, uint32_t HR,
                               uint32_t bin_size, uint32_t* splits, PartDesc* rdesc, hipStream_t s) {
  k_range_splits<<<1, kBlock, 0, s>>>(bin_offset, nbins, n, P, HR, bin_size, splits, rdesc);
  return hipGetLastError();
}

hipError_t launch_layout(const uint32_t* tile_base, uint32_t num_tiles, uint32_t P, uint32_t n, uint32_t num,
                         uint32_t den, uint64_t V_plain, uint32_t* part_offsets, uint32_t* bucket_base,
                         PartDesc* desc, hipStream_t s) {
  k_layout<<<1, kBlock, 0, s>>>(tile_base, num_tiles, P, n, num, den, V_plain, part_offsets, bucket_base, desc);
  return hipGetLastError();
}

hipError_t launch_hist(int kt, const void* keys, uint32_t n, uint32_t log2P, uint32_t P, const PartDesc* desc,
                       uint32_t* cnt, hipStream_t s) {
  const uint32_t tiles = div_up(n, kTileKeys);
  if (tiles == 0) return hipSuccess;
  if (kt == 0)
    k_hist<uint32_t><<<tiles, kBlock, 0, s>>>(static_cast<const uint32_t*>(keys), n, log2P, P, desc, cnt);
  else
    k_hist<uint64_t><<<tiles, kBlock, 0, s>>>(static_cast<const uint64_t*>(keys), n, log2P, P, desc, cnt);
  return hipGetLastError();
}

hipError_t launch_scatter(int kt, const void* keys, uint32_t n, uint32_t log2P, uint32_t P, const PartDesc* desc,
                          uint32_t* cursor, void* out, hipStream_t s) {
  const uint32_t tiles = div_up(n, kTileKeys);
  if (tiles == 0) return hipSuccess;
  if (kt == 0)
    k_scatter<uint32_t><<<tiles, kBlock, 0, s>>>(static_cast<const uint32_t*>(keys), n, log2P, P, desc, cursor,
                                                 static_cast<uint32_t*>(out));
  else
    k_scatter<uint64_t><<<tiles, kBlock, 0, s>>>(static_cast<const uint64_t*>(keys), n, log2P, P, desc, cursor,
                                                 static_cast<uint64_t*>(out));
  return hipGetLastError();
}

hipError_t launch_probe(int kt, bool count, const void* tkeys, const uint32_t* offsets, const PartDesc* desc,
                        uint32_t log2P, uint32_t P, const uint32_t* unsorted, const void* queries, uint32_t q,
                        void* out, hipStream_t s) {
  const uint32_t tiles = div_up(q, kTileKeys);
  if (tiles == 0) return hipSuccess;
  if (kt == 0) {
    const uint32_t* tk = static_cast<const uint32_t*>(tkeys);
    const uint32_t* qs = static_cast<const uint32_t*>(queries);
    if (count)
      k_probe<uint32_t, true><<<tiles, kBlock, 0, s>>>(tk, offsets, desc, log2P, P, unsorted, qs, q, out);
    else
      k_probe<uint32_t, false><<<tiles, kBlock, 0, s>>>(tk, offsets, desc, log2P, P, unsorted, qs, q, out);
  } else {
    const uint64_t* tk = static_cast<const uint64_t*>(tkeys);
    const uint64_t* qs = static_cast<const uint64_t*>(queries);
    if (count)
      k_probe<uint64_t, true><<<tiles, kBlock, 0, s>>>(tk, offsets, desc, log2P, P, unsorted, qs, q, out);
    else
      k_probe<uint64_t, false><<<tiles, kBlock, 0, s>>>(tk, offsets, desc, log2P, P, unsorted, qs, q, out);
  }
  return hipGetLastError();
}

hipError_t launch_hash_bucket(int kt, const void* keys, uint32_t n, uint32_t V, uint64_t* hash, uint32_t* bucket,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  const PartDesc d = make_desc(V, 0);
  if (kt == 0)
    k_hash_bucket<uint32_t><<<grid_for(n), kBlock, 0, s>>>(static_cast<const uint32_t*>(keys), n, d, hash, bucket);
  else
    k_hash_bucket<uint64_t><<<grid_for(n), kBlock, 0, s>>>(static_cast<const uint64_t*>(keys), n, d, hash, bucket);
  return hipGetLastError();
}

}  // namespace hg
