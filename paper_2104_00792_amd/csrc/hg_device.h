// Device-side building blocks of the HashGraph path on gfx950.
//
// Hash: MurmurHash3 finalizers on the key value (fmix32 / fmix64; the paper
// names Murmur in Sec. 4.2).  Bucket: a true remainder hash mod V
// (Algorithm 1, first loop), computed without a divide instruction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

constexpr int kWave = 64;

// ---------------------------------------------------------------- hashing
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

__host__ __device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

template <typename K> struct KeyTraits;
template <> struct KeyTraits<uint32_t> {
  typedef uint32_t Hash;
  static constexpr int kBits = 32;
  __host__ __device__ static __forceinline__ uint32_t hash(uint32_t k) { return fmix32(k); }
};
template <> struct KeyTraits<uint64_t> {
  typedef uint64_t Hash;
  static constexpr int kBits = 64;
  __host__ __device__ static __forceinline__ uint64_t hash(uint64_t k) { return fmix64(k); }
};

// Partition of a hash: its top log2P bits (0 when log2P == 0).
// One bit-field extract of the hash's upper word: a field of width 0 is 0,
// so P == 1 needs no separate case.  P <= 256: the mask states the range,
// which lets the compiler index the 24-byte descriptors with shifts and
// adds instead of a quarter-rate multiply.
template <typename H>
__device__ __forceinline__ uint32_t part_of(H h, uint32_t log2P) {
  const uint32_t hi = static_cast<uint32_t>(h >> (sizeof(H) * 8 - 32));
  return __builtin_amdgcn_ubfe(hi, (32u - log2P) & 31u, log2P) & 0xFFu;
}

// ------------------------------------------------------------ bucket map
// h mod V by a truncated reciprocal.  With m = floor((2^w - 1) / V) the
// estimate q = floor(h * m / 2^w) satisfies floor(h/V) - 1 <= q <= floor(h/V)
// (h * m / 2^w lies in (h/V - 1, h/V)), so r = h - q*V lies in [0, 2V) and one
// conditional subtraction gives the exact remainder.  r never exceeds h, so
// no intermediate overflows.
__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b) {
  return static_cast<uint32_t>((static_cast<uint64_t>(a) * b) >> 32);
}

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) {
  return static_cast<uint64_t>((static_cast<unsigned __int128>(a) * b) >> 64);
}

__host__ __device__ __forceinline__ uint32_t recip32(uint32_t V) { return 0xFFFFFFFFu / V; }
__host__ __device__ __forceinline__ uint64_t recip64(uint32_t V) { return ~0ull / V; }

// floor(h / V) by the same truncated reciprocal (one correction step).
__host__ __device__ __forceinline__ uint32_t quot_by_recip(uint32_t h, uint32_t V, uint32_t m32) {
  const uint32_t q = mulhi32(h, m32);
  return h - q * V >= V ? q + 1 : q;
}

__host__ __device__ __forceinline__ uint32_t mod_by_recip(uint32_t h, uint32_t V, uint32_t m32, uint64_t) {
  const uint32_t q = mulhi32(h, m32);
  const uint32_t r = h - q * V;
  // r < 2V and r <= h < 2^32: when r < V, r - V wraps to r + 2^32 - V > r,
  // so the smaller of the two is the remainder either way (a subtract and a
  // min instead of a compare, a select and a subtract).
  const uint32_t s = r - V;
  return s < r ? s : r;
}

__host__ __device__ __forceinline__ uint32_t mod_by_recip(uint64_t h, uint32_t V, uint32_t, uint64_t m64) {
  const uint64_t q = mulhi64(h, m64);
  uint64_t r = h - q * static_cast<uint64_t>(V);
  return static_cast<uint32_t>(r >= V ? r - V : r);
}

// Per-partition table descriptor: table size, first global bucket, the two
// reciprocals of the bucket map, and pmask = V - 1 when V is a power of two
// (then hash mod V is the hash's low bits), else kNotPow2.
constexpr uint32_t kNotPow2 = 0xFFFFFFFFu;
struct PartDesc {
  uint32_t V;
  uint32_t base;
  uint32_t m32;
  uint32_t pmask;
  uint64_t m64;
};

__host__ __device__ __forceinline__ PartDesc make_desc(uint32_t V, uint32_t base) {
  PartDesc d;
  d.V = V;
  d.base = base;
  d.m32 = recip32(V);
  d.pmask = (V & (V - 1u)) == 0u ? V - 1u : kNotPow2;  // V >= 1
  d.m64 = recip64(V);
  return d;
}

// Global bucket of a hash under descriptor d: the low bits for a table size
// that is a power of two (no multiply), else the remainder by reciprocal.
// Both give hash mod V exactly.
template <typename H>
__device__ __forceinline__ uint32_t global_bucket(H h, const PartDesc& d) {
  if (d.pmask != kNotPow2) return d.base + (static_cast<uint32_t>(h) & d.pmask);
  return d.base + mod_by_recip(h, d.V, d.m32, d.m64);
}

// ------------------------------------------------------ wave primitives
__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return static_cast<uint32_t>(__popcll(m)); }

__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t lane) {
  return __builtin_amdgcn_readlane(v, lane);
}

// A value that every lane of the wave holds alike (say one LDS word that all
// lanes read), taken from the first active lane.  The compiler then knows it
// is wave-uniform: branches and loop exits that depend on it stay scalar, so
// the wave is never split between the paths of a loop.  Without it, a loop
// whose exit depends on an LDS load is compiled with per-lane exit masks, and
// lanes may re-enter the loop while others wait at its exit; a value one lane
// computes and readlane broadcasts is then read while that lane is away.
__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Inclusive sum over the 64 lanes of a wave with DPP lane moves (no LDS
// round trip): shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the
// last lane of a row is broadcast into the next row (row_bcast:15 into rows 1
// and 3) and lane 31 into rows 2 and 3 (row_bcast:31).  Lanes with no source
// receive 0 (the `old` operand).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_or_zero(uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), kCtrl, kRowMask, 0xF, false));
}

__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
  constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
  v += dpp_or_zero<kRowShr + 1, 0xF>(v);
  v += dpp_or_zero<kRowShr + 2, 0xF>(v);
  v += dpp_or_zero<kRowShr + 4, 0xF>(v);
  v += dpp_or_zero<kRowShr + 8, 0xF>(v);
  v += dpp_or_zero<kRowBcast15, 0xA>(v);
  v += dpp_or_zero<kRowBcast31, 0xC>(v);
  return v;
}

// ------------------------------------------------------ bucket counting
// Whether long bucket g is known to be sorted (see the table's unsorted
// block: word 0 = number of unsorted long buckets, then their ids).
__device__ __forceinline__ bool long_bucket_sorted(const uint32_t* unsorted, uint32_t nunsorted, uint32_t g,
                                                   uint32_t max_listed) {
  if (nunsorted == 0) return true;
  if (nunsorted > max_listed) return false;
  for (uint32_t i = 0; i < nunsorted; ++i)
    if (unsorted[1 + i] == g) return false;
  return true;
}

// Occurrences of q among the keys a[lo, hi) of a short bucket held in LDS.
// Keys are read four at a time whatever the bucket's length (a[] has four
// spare entries past its last key) and masked by it, so the common bucket of
// a few keys costs two paired LDS reads and no loop, and a longer one (up to
// kLongT keys, a table with many keys per bucket) a quarter of the dependent
// rounds of a key-by-key loop.
template <typename K>
__device__ __forceinline__ uint32_t count_short(const K* a, uint32_t lo, uint32_t hi, K q) {
  const uint32_t n = hi - lo;
  const K x0 = a[lo], x1 = a[lo + 1], x2 = a[lo + 2], x3 = a[lo + 3];
  uint32_t c = (x0 == q && n > 0 ? 1u : 0u) + (x1 == q && n > 1 ? 1u : 0u) + (x2 == q && n > 2 ? 1u : 0u) +
               (x3 == q && n > 3 ? 1u : 0u);
  for (uint32_t x = lo + 4; x < hi; x += 4) {
    const K y0 = a[x], y1 = a[x + 1], y2 = a[x + 2], y3 = a[x + 3];
    c += (y0 == q ? 1u : 0u) + (y1 == q && x + 1 < hi ? 1u : 0u) + (y2 == q && x + 2 < hi ? 1u : 0u) +
         (y3 == q && x + 3 < hi ? 1u : 0u);
  }
  return c;
}

// Occurrences of q among a[lo, hi): a linear scan, or, when the range is
// sorted, a look at its two ends and at most two binary searches.
template <typename K, typename Ptr>
__device__ __forceinline__ uint32_t count_equal(Ptr a, uint32_t lo, uint32_t hi, K q, bool sorted) {
  if (!sorted) {
    uint32_t c = 0;
    for (uint32_t x = lo; x < hi; ++x) c += a[x] == q ? 1u : 0u;
    return c;
  }
  if (lo >= hi) return 0;
  // Both ends in one round trip: a bucket of one value (a heavy key alone
  // in its bucket, the common long bucket of a skewed table) or a query
  // outside the bucket's range needs no search.
  const K first = a[lo], last = a[hi - 1];
  if (first == last) return first == q ? hi - lo : 0u;
  if (q < first || q > last) return 0;
  uint32_t l = lo, h = hi;  // first position with a[x] >= q
  if (first != q) {
    while (l < h) {
      const uint32_t mid = l + ((h - l) >> 1);
      if (a[mid] < q) l = mid + 1; else h = mid;
    }
  }
  uint32_t u = hi, uh = hi;  // first position with a[x] > q
  if (last != q) {
    u = l;
    while (u < uh) {
      const uint32_t mid = u + ((uh - u) >> 1);
      if (a[mid] <= q) u = mid + 1; else uh = mid;
    }
  }
  return u - l;
}

}  // namespace hg
