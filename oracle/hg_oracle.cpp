// HashGraph CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
//
// Only the test suite, the smoke check and the benchmark's CPU-baseline leg
// may load this library.  The GPU library never links, includes or calls it,
// and it shares no code with the GPU path: every function here is written
// from the definitions in the paper (Tripathy & Green, "Scalable Hash Table
// for NUMA Systems", arXiv 2104.00792) in the plainest form available:
// std::sort of tuples plus run-length counting.
//
// What is computed (Sec. 3.1 "Single-GPU HashGraph", Algorithm 1; Sec. 3.3
// Phase 2, Algorithm 2; the CSR paragraph of Sec. 3.1; the count-balanced
// ranges of Algorithm 2, Phase 1, in step O6 below):
//   * hash(e): the MurmurHash3 64/32-bit finalizers applied to the key value
//     (Sec. 4.2 names Murmur; the variant is our reading, see below).
//   * partition of a key: the top log2(P) bits of its hash (fixed equal hash
//     ranges, Sec. 3.3 "Phase 1" with equal splits).
//   * table size of partition p: V_p = max(1, floor(n_p * num / den)), i.e.
//     V = N / C with C = den / num (Sec. 2, Algorithm 1 caption), unless an
//     explicit bucket count is given for a plain (P = 1) table.
//   * bucket of a key: hash mod V_p (Algorithm 1, first loop).
//   * offset[g] = number of keys whose global bucket is < g, where the global
//     bucket is bucket_base[p] + b and bucket_base is the prefix sum of V_p;
//     offset[sum V_p] = n (CSR offset array, Sec. 3.1).
//   * keys[offset[g] .. offset[g+1]) = the keys of bucket g, listed here in
//     ascending order (the canonical form; the paper leaves the order inside
//     a bucket to the atomics of Algorithm 1).
//   * count(x) = number of i with A[i] == x (Sec. 5.4: the query counts how
//     many times each key appears); found(x) = count(x) > 0 (Sec. 3.3
//     "Querying").
//
// Readings of the paper that this file commits to (each also in the design
// notes): Murmur = fmix32 / fmix64 finalizers, unseeded; bucket = true
// remainder (never a multiply-shift range reduction); partitions by the top
// hash bits; V_p >= 1 always; n = 0 is a legal empty table.
//
// Threads.  Built plainly (g++ -O2) every loop runs on one thread.  The
// all-core build compiles this same file with -fopenmp -D_GLIBCXX_PARALLEL:
// std::sort then runs as the GNU parallel-mode sort, and the two loops
// marked `omp parallel for` (independent iterations, each writing only its
// own element) are shared among the threads.  Nothing else changes.
//
// Pins (what ties this file to something other than itself) live in the
// test suite: published MurmurHash3 test vectors and a library MurmurHash3
// for fmix32, SMHasher's published verification value of MurmurHash3_x64_128
// for fmix64, Python-integer remainders for the bucket map, brute force on
// tiny inputs for the CSR, and invariants at every size.

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <tuple>
#include <vector>

namespace {

// MurmurHash3 32-bit finalizer (fmix32), applied to the key value.
inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// MurmurHash3 64-bit finalizer (fmix64), applied to the key value.
inline uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

enum { KT_U32 = 0, KT_U64 = 1 };
enum { ORC_OK = 0, ORC_BAD_ARG = 1, ORC_TOO_BIG = 2 };

inline uint64_t key_at(const void* keys, int kt, uint64_t i) {
  return kt == KT_U32 ? static_cast<const uint32_t*>(keys)[i]
                      : static_cast<const uint64_t*>(keys)[i];
}

inline void key_put(void* keys, int kt, uint64_t i, uint64_t v) {
  if (kt == KT_U32)
    static_cast<uint32_t*>(keys)[i] = static_cast<uint32_t>(v);
  else
    static_cast<uint64_t*>(keys)[i] = v;
}

// hash(e): 32-bit keys use fmix32, 64-bit keys use fmix64.
inline uint64_t hash_of(uint64_t key, int kt) {
  return kt == KT_U32 ? fmix32(static_cast<uint32_t>(key)) : fmix64(key);
}

inline uint32_t log2_exact(uint32_t P) {
  uint32_t l = 0;
  while ((1u << l) < P) ++l;
  return l;
}

// Partition of a hashed key: the top log2(P) bits of the hash word.
inline uint32_t part_of(uint64_t h, int kt, uint32_t log2P) {
  if (log2P == 0) return 0;
  const uint32_t w = kt == KT_U32 ? 32 : 64;
  return static_cast<uint32_t>(h >> (w - log2P));
}

bool valid_common(uint64_t n, int kt, uint32_t P) {
  if (kt != KT_U32 && kt != KT_U64) return false;
  if (n >= (1ull << 32)) return false;
  if (P == 0 || (P & (P - 1)) != 0 || P > 65536) return false;
  return true;
}

// Table size of every partition: V_p = max(1, floor(n_p * num / den)),
// or the explicit bucket count for a plain table.  Returns false when the
// total bucket count does not fit the 32-bit offset array.
bool table_sizes(const std::vector<uint64_t>& n_p, uint32_t P, uint32_t num,
                 uint32_t den, uint64_t V_plain, std::vector<uint64_t>& V) {
  V.assign(P, 0);
  uint64_t total = 0;
  for (uint32_t p = 0; p < P; ++p) {
    uint64_t v;
    if (P == 1 && V_plain != 0) {
      v = V_plain;
    } else {
      // n_p < 2^32 and num < 2^32, so the product fits in 64 bits.
      v = n_p[p] * static_cast<uint64_t>(num) / den;
      if (v < 1) v = 1;
    }
    V[p] = v;
    total += v;
    if (total > 0xFFFFFFFEull) return false;
  }
  return true;
}

}  // namespace

extern "C" {

uint32_t orc_fmix32(uint32_t h) { return fmix32(h); }
uint64_t orc_fmix64(uint64_t k) { return fmix64(k); }

// hash(A[i]) and hash(A[i]) mod V for a single table size V (Algorithm 1,
// first loop).  hash_out or bucket_out may be null.
int orc_hash_bucket(const void* keys, uint64_t n, int kt, uint64_t V,
                    uint64_t* hash_out, uint32_t* bucket_out) {
  if ((kt != KT_U32 && kt != KT_U64) || V == 0 || V > 0xFFFFFFFFull)
    return ORC_BAD_ARG;
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t h = hash_of(key_at(keys, kt, i), kt);
    if (hash_out) hash_out[i] = h;
    if (bucket_out) bucket_out[i] = static_cast<uint32_t>(h % V);
  }
  return ORC_OK;
}

// Partition sizes and table sizes only: part_offsets[P+1] (exclusive prefix
// of n_p) and bucket_base[P+1] (exclusive prefix of V_p; bucket_base[P] is
// the total bucket count).  Lets a caller size the offset array.
int orc_layout(const void* keys, uint64_t n, int kt, uint32_t P, uint32_t num,
               uint32_t den, uint64_t V_plain, uint32_t* part_offsets,
               uint32_t* bucket_base) {
  if (!valid_common(n, kt, P)) return ORC_BAD_ARG;
  if (!(P == 1 && V_plain != 0) && (num == 0 || den == 0)) return ORC_BAD_ARG;
  const uint32_t log2P = log2_exact(P);
  std::vector<uint64_t> n_p(P, 0);
  for (uint64_t i = 0; i < n; ++i)
    ++n_p[part_of(hash_of(key_at(keys, kt, i), kt), kt, log2P)];
  std::vector<uint64_t> V;
  if (!table_sizes(n_p, P, num, den, V_plain, V)) return ORC_TOO_BIG;
  uint64_t po = 0, bb = 0;
  for (uint32_t p = 0; p < P; ++p) {
    part_offsets[p] = static_cast<uint32_t>(po);
    bucket_base[p] = static_cast<uint32_t>(bb);
    po += n_p[p];
    bb += V[p];
  }
  part_offsets[P] = static_cast<uint32_t>(po);
  bucket_base[P] = static_cast<uint32_t>(bb);
  return ORC_OK;
}

// The whole build, steps O1-O3:
//   O1  h = hash(A[i]); p = top bits of h; n_p; V_p; b = h mod V_p
//   O2  std::sort of the tuples (p, b, A[i]) in lexicographic order
//   O3  run-length counts of p and of (p, b), exclusive prefix sums
// Outputs: part_offsets[P+1], bucket_base[P+1], offsets[sum V_p + 1] (the
// caller sizes it with orc_layout), keys_out[n] (canonical: each bucket
// ascending).
int orc_build(const void* keys, uint64_t n, int kt, uint32_t P, uint32_t num,
              uint32_t den, uint64_t V_plain, uint32_t* part_offsets,
              uint32_t* bucket_base, uint32_t* offsets, uint64_t offsets_cap,
              void* keys_out) {
  if (!valid_common(n, kt, P)) return ORC_BAD_ARG;
  if (!(P == 1 && V_plain != 0) && (num == 0 || den == 0)) return ORC_BAD_ARG;
  const uint32_t log2P = log2_exact(P);

  // O1: hash, partition, partition sizes.
  std::vector<uint64_t> h(n);
  std::vector<uint32_t> p_of(n);
  std::vector<uint64_t> n_p(P, 0);
  for (uint64_t i = 0; i < n; ++i) {
    h[i] = hash_of(key_at(keys, kt, i), kt);
    p_of[i] = part_of(h[i], kt, log2P);
    ++n_p[p_of[i]];
  }
  std::vector<uint64_t> V;
  if (!table_sizes(n_p, P, num, den, V_plain, V)) return ORC_TOO_BIG;
  uint64_t total_buckets = 0;
  for (uint32_t p = 0; p < P; ++p) total_buckets += V[p];
  if (offsets_cap < total_buckets + 1) return ORC_BAD_ARG;

  // O1 (cont.): the bucket of every key inside its partition's table.
  typedef std::tuple<uint32_t, uint32_t, uint64_t> Tup;  // (p, b, key)
  std::vector<Tup> t(n);
#pragma omp parallel for schedule(static)
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t b = static_cast<uint32_t>(h[i] % V[p_of[i]]);
    t[i] = Tup(p_of[i], b, key_at(keys, kt, i));
  }

  // O2: one lexicographic sort puts partitions, buckets and keys in order.
  std::sort(t.begin(), t.end());

  // O3: run-length counts and exclusive prefix sums.
  uint64_t bb = 0, po = 0;
  for (uint32_t p = 0; p < P; ++p) {
    bucket_base[p] = static_cast<uint32_t>(bb);
    part_offsets[p] = static_cast<uint32_t>(po);
    bb += V[p];
    po += n_p[p];
  }
  bucket_base[P] = static_cast<uint32_t>(bb);
  part_offsets[P] = static_cast<uint32_t>(po);

  std::vector<uint32_t> bucket_count(total_buckets, 0);
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t g = bucket_base[std::get<0>(t[i])] + std::get<1>(t[i]);
    ++bucket_count[g];
    key_put(keys_out, kt, i, std::get<2>(t[i]));
  }
  uint64_t run = 0;
  for (uint64_t g = 0; g < total_buckets; ++g) {
    offsets[g] = static_cast<uint32_t>(run);
    run += bucket_count[g];
  }
  offsets[total_buckets] = static_cast<uint32_t>(run);
  return ORC_OK;
}

// Step O4: exact multiplicity of every query in A, from a sorted copy of A
// and equal_range.  Independent of the hash, of V and of P.
int orc_count(const void* keys, uint64_t n, int kt, const void* queries,
              uint64_t q, uint32_t* counts) {
  if (kt != KT_U32 && kt != KT_U64) return ORC_BAD_ARG;
  if (n >= (1ull << 32)) return ORC_BAD_ARG;
  std::vector<uint64_t> a(n);
  for (uint64_t i = 0; i < n; ++i) a[i] = key_at(keys, kt, i);
  std::sort(a.begin(), a.end());
#pragma omp parallel for schedule(static)
  for (uint64_t j = 0; j < q; ++j) {
    const uint64_t x = key_at(queries, kt, j);
    const auto r = std::equal_range(a.begin(), a.end(), x);
    counts[j] = static_cast<uint32_t>(r.second - r.first);
  }
  return ORC_OK;
}

// Step O5: the partition split alone (Algorithm 2, Phase 2 with fixed equal
// hash ranges).  part_offsets[P+1]; keys_out holds each partition's keys in
// ascending order (the paper leaves the order inside a partition open).
int orc_bin_partition(const void* keys, uint64_t n, int kt, uint32_t P,
                      uint32_t* part_offsets, void* keys_out) {
  if (!valid_common(n, kt, P)) return ORC_BAD_ARG;
  const uint32_t log2P = log2_exact(P);
  std::vector<std::pair<uint32_t, uint64_t>> t(n);
  std::vector<uint64_t> n_p(P, 0);
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t k = key_at(keys, kt, i);
    const uint32_t p = part_of(hash_of(k, kt), kt, log2P);
    t[i] = std::make_pair(p, k);
    ++n_p[p];
  }
  std::sort(t.begin(), t.end());
  uint64_t po = 0;
  for (uint32_t p = 0; p < P; ++p) {
    part_offsets[p] = static_cast<uint32_t>(po);
    po += n_p[p];
  }
  part_offsets[P] = static_cast<uint32_t>(po);
  for (uint64_t i = 0; i < n; ++i) key_put(keys_out, kt, i, t[i].second);
  return ORC_OK;
}

// Step O6: the count-balanced split of Algorithm 2, Phases 1 and 2 (Sec. 3.3,
// "Phase 1: Multi-GPU Data Partitioning" and "Phase 2"), one partition per
// device.  The reduced hash H = hash mod HR covers the hash range HR; the
// range is cut into bins of BinSize = ceil(HR / num_bins) consecutive values
// (bin = floor(H / BinSize), ceil(HR / BinSize) bins; num_bins = 0 takes
// ceil(sqrt(HR)), at most 2^14).  BinOffset is the exclusive prefix sum of the
// keys per bin.  Boundary d (0 < d < P) is the first bin whose BinOffset
// reaches floor(n * d / P), the key count the first d partitions should hold;
// split[0] = 0 and split[P] = the number of bins.  A key belongs to the last
// partition d with split[d] <= bin.  Outputs: part_offsets[P+1], bin_splits
// [P+1], and the keys grouped by partition, each group ascending.
int orc_bin_partition_balanced(const void* keys, uint64_t n, int kt, uint32_t P, uint64_t HR, uint32_t num_bins,
                               uint32_t* part_offsets, uint32_t* bin_splits, void* keys_out) {
  if (kt != KT_U32 && kt != KT_U64) return ORC_BAD_ARG;
  if (n >= (1ull << 32) || P == 0 || P > 256 || HR == 0 || HR >= (1ull << 32) || num_bins > (1u << 14))
    return ORC_BAD_ARG;
  uint64_t bins_asked = num_bins;
  if (bins_asked == 0) {
    bins_asked = 1;
    while (bins_asked * bins_asked < HR) ++bins_asked;  // ceil(sqrt(HR))
    if (bins_asked > (1u << 14)) bins_asked = 1u << 14;
  }
  const uint64_t bin_size = (HR + bins_asked - 1) / bins_asked;
  const uint64_t nbins = (HR + bin_size - 1) / bin_size;
  std::vector<uint64_t> bin_of(n);
  std::vector<uint64_t> count(nbins, 0);
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t H = hash_of(key_at(keys, kt, i), kt) % HR;
    bin_of[i] = H / bin_size;
    ++count[bin_of[i]];
  }
  std::vector<uint64_t> bin_offset(nbins + 1, 0);
  for (uint64_t b = 0; b < nbins; ++b) bin_offset[b + 1] = bin_offset[b] + count[b];
  std::vector<uint64_t> split(P + 1, 0);
  split[P] = nbins;
  for (uint32_t d = 1; d < P; ++d) {
    const uint64_t target = n * d / P;
    split[d] = static_cast<uint64_t>(std::lower_bound(bin_offset.begin(), bin_offset.end(), target) -
                                     bin_offset.begin());
  }
  std::vector<std::pair<uint32_t, uint64_t>> t(n);
  std::vector<uint64_t> n_d(P, 0);
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t d =
        static_cast<uint32_t>(std::upper_bound(split.begin(), split.end(), bin_of[i]) - split.begin()) - 1;
    t[i] = std::make_pair(d, key_at(keys, kt, i));
    ++n_d[d];
  }
  std::sort(t.begin(), t.end());
  uint64_t po = 0;
  for (uint32_t d = 0; d < P; ++d) {
    part_offsets[d] = static_cast<uint32_t>(po);
    po += n_d[d];
  }
  part_offsets[P] = static_cast<uint32_t>(po);
  for (uint32_t d = 0; d <= P; ++d) bin_splits[d] = static_cast<uint32_t>(split[d]);
  for (uint64_t i = 0; i < n; ++i) key_put(keys_out, kt, i, t[i].second);
  return ORC_OK;
}

}  // extern "C"
