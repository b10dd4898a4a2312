// The LDS-sorted HashGraph path for gfx950.
//
// Algorithm 1 of Tripathy & Green (arXiv 2104.00792) counts keys per hash
// value, prefix-sums the counts and scatters the keys with atomics at random
// addresses.  At 2^28 keys those random accesses miss every cache; here the
// same result is reached with streaming passes only:
//   level-1 split  by partition (Algorithm 2, Phase 2) or by coarse bucket
//                  range: per-tile counts + scan + scatter;
//   level-2 split  by sub-bin of up to 2^13 buckets inside each level-1
//                  segment (the paper's second, local binning for cache
//                  locality, Sec. 3.2, sized here for the LDS of a CU);
//   LDS build      one workgroup per sub-bin: histogram, exclusive scan and
//                  scatter of Algorithm 1, all three in LDS.
// A split ranks the keys of a tile by one LDS atomic each on the tile's
// histogram, like the atomic scatter of Algorithm 1: the order inside a
// digit is whatever the atomics give, which the table leaves free.
// Queries follow the same two splits, recording where each query went, are
// counted against LDS-resident windows of the table, and return to their
// input order by two gathers through those permutations.
#include <type_traits>

#include "hg_internal.h"
#include "hg_tile.h"

namespace hg {
namespace {

template <typename K>
__device__ __forceinline__ uint32_t bucket_of(K key, uint32_t log2P, const PartDesc* sd) {
  const auto h = KeyTraits<K>::hash(key);
  return global_bucket(h, sd[part_of(h, log2P)]);
}

// x must be in registers here: a load issued above cannot sink below this
// point (the compiler otherwise moves loads down to their first use, past
// barriers they do not depend on, and the workgroup pays two round trips
// instead of one).
template <typename T>
__device__ __forceinline__ void in_regs(T& x) {
  asm volatile("" : "+v"(x));
}

// Adds add (0 or 1) to h[idx] for every lane of the wave; with kReturn each
// lane with add = 1 gets a distinct old value (its rank).  LDS serves the
// lanes of one atomic that hit one address one after another, so a wave of
// mostly equal indexes (many copies of one key) would take 64 turns.  While
// the first lane not yet served shares its index with at least kHistGroup
// lanes (for up to kHistRounds indexes), those lanes add their sum with one
// atomic; the rest add their own.  The grouping costs a few instructions
// per call and, with kReturn, a wait for each atomic's result, so callers
// take this path only for waves that wave_skewed flags.
constexpr uint32_t kHistGroup = 8;
constexpr int kHistRounds = 3;
constexpr uint32_t kSkewLanes = 16;

// Whether at least kSkewLanes active lanes hold the first active lane's idx
// (wave-uniform): one sample per wave decides which histogram path the wave
// takes for all its items.
__device__ __forceinline__ bool wave_skewed(uint32_t idx) {
  return popc64(ballot(idx == wave_uniform(idx))) >= kSkewLanes;
}

template <bool kReturn>
__device__ __forceinline__ uint32_t lds_hist_add(uint32_t* h, uint32_t idx, uint32_t add) {
  uint32_t pos = 0;
  bool done = false;
#pragma unroll
  for (int r = 0; r < kHistRounds; ++r) {
    const uint64_t rest = ballot(!done);
    if (rest == 0) break;
    const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(rest)) - 1);
    const uint32_t li = readlane(idx, leader);
    const bool in = !done && idx == li;
    const uint64_t same = ballot(in);
    if (popc64(same) < kHistGroup) break;
    const uint64_t adds = ballot(in && add != 0);
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(&h[li], popc64(adds));
    if (kReturn) {
      base = readlane(base, leader);
      if (in) pos = base + popc64(adds & lanemask_lt());
    }
    done = done || in;
  }
  if (!done && (kReturn || add != 0)) {
    const uint32_t p = atomicAdd(&h[idx], add);
    if (kReturn) pos = p;
  }
  return pos;
}

// p[i] for a wave-uniform i, where p points into an array that earlier
// launches wrote and this one only reads (the plan's arrays and scanned
// counts).  The pointer is taken as a constant-address-space pointer, so
// the load is a scalar one: the plan's arrays are reached through pointers
// stored in the plan, and read as generic pointers they become per-wave
// vector (flat) loads, two dependent round trips before any work starts.
__device__ __forceinline__ uint32_t ld_uniform(const uint32_t* p, uint32_t i) {
  typedef __attribute__((address_space(4))) const uint32_t ConstU32;
  const ConstU32* q = reinterpret_cast<const ConstU32*>(reinterpret_cast<uintptr_t>(p));
  return q[wave_uniform(i)];
}

// Index of the last segment whose prefix value is <= x (arr[0] == 0, arr is
// non-decreasing over 0..nseg).
__device__ __forceinline__ uint32_t find_segment(const uint32_t* arr, uint32_t nseg, uint32_t x) {
  uint32_t lo = 0, hi = nseg;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (arr[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------ multisplit
// Item i of thread t holds element elem(i, t) of its tile: with 16-byte loads
// (a whole, aligned tile) thread t reads kVec consecutive keys per load;
// otherwise one key per load, striped over the workgroup.  Both passes over a
// tile take the same branch, so their orders agree.
template <typename K, int THREADS>
__device__ __forceinline__ uint32_t elem_of(bool vec, int i, uint32_t t) {
  constexpr int kVec = 16 / sizeof(K);
  return vec ? (static_cast<uint32_t>(i / kVec) * THREADS + t) * kVec + static_cast<uint32_t>(i % kVec)
             : static_cast<uint32_t>(i) * THREADS + t;
}

// Loads the keys of a tile: elements base + e for head <= e < tail.  With
// `vec` (a whole tile at a 16-byte aligned base) thread t reads kVec
// consecutive keys per load.  Items outside the tile hold key 0.
template <typename K, int THREADS, int ITEMS>
__device__ __forceinline__ uint32_t load_items(const K* __restrict__ in, uint32_t base, uint32_t head, uint32_t tail,
                                               bool vec, K (&v)[ITEMS]) {
  constexpr int kVec = 16 / sizeof(K);
  const uint32_t t = threadIdx.x;
  if (vec) {
    const uint4* p = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
    for (int j = 0; j < ITEMS / kVec; ++j) {
      const uint4 x = p[j * THREADS + t];
      K tmp[kVec];
      __builtin_memcpy(tmp, &x, 16);
#pragma unroll
      for (int c = 0; c < kVec; ++c) v[j * kVec + c] = tmp[c];
    }
    return ITEMS == 32 ? 0xFFFFFFFFu : ((1u << ITEMS) - 1u);
  }
  uint32_t mask = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t e = static_cast<uint32_t>(i) * THREADS + t;
    v[i] = K(0);  // items past the tile hold a harmless key
    if (e >= head && e < tail) {
      v[i] = in[base + e];
      mask |= 1u << i;
    }
  }
  return mask;
}

// Workgroups reach the 8 XCDs of the chip round robin (workgroup b runs on
// XCD b % 8), and each XCD has its own L2.  Tile numbers are reassigned so
// that every XCD walks one contiguous range of tiles in order: neighbouring
// tiles write neighbouring pieces of each digit run and of each count row,
// and those partial lines now meet in one L2 instead of leaving it half
// written.  A bijection of [0, G).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t G) {
  constexpr uint32_t kXcd = 8;
  const uint32_t q = G / kXcd, r = G % kXcd, x = b % kXcd;
  return x * q + min(x, r) + b / kXcd;
}

// Where split tile blockIdx.x lies: its segment (plan) or the single segment
// [0, n) with nd digits and gridDim.x tiles, the digit count D, the tiles T
// and count base cb of the segment, and the tile's keys [base + head, base +
// tail).  The tiles of a segment start at its first key rounded down to
// kTileAlign keys, so that every interior tile takes 16-byte loads; the first
// and last tiles mask what lies outside the segment.  False: no tile (the
// workgroup exits).
struct TileLoc {
  uint32_t D, T, k0, k1, cb, gs, tl, seg, base, head, tail;
};

__device__ __forceinline__ bool tile_loc(const SegPlan* plan, uint32_t nd, uint32_t n, uint32_t tile, TileLoc& L) {
  L.D = nd;
  L.T = gridDim.x;
  L.k0 = 0;
  L.k1 = n;
  L.cb = 0;
  L.gs = 0;
  L.seg = 0;
  if (plan != nullptr) {
    const uint32_t G = plan->total_tiles;
    if (blockIdx.x >= G) return false;
    const uint32_t b = xcd_tile(blockIdx.x, G);
    L.seg = ld_uniform(plan->tile_seg, b);
    L.tl = b - ld_uniform(plan->tile_first, L.seg);
    L.D = ld_uniform(plan->D, L.seg);
    L.T = ld_uniform(plan->T, L.seg);
    L.k0 = ld_uniform(plan->key0, L.seg);
    L.k1 = ld_uniform(plan->key0, L.seg + 1);
    L.cb = ld_uniform(plan->cbase, L.seg);
    L.gs = ld_uniform(plan->g0, L.seg);
  } else {
    L.tl = xcd_tile(blockIdx.x, gridDim.x);
  }
  L.base = (L.k0 & ~(kTileAlign - 1)) + L.tl * tile;
  L.head = L.base < L.k0 ? L.k0 - L.base : 0u;
  L.tail = min(tile, L.k1 - L.base);
  return true;
}

// One split pass over a tile: per-tile digit counts (COUNT), or the move of
// the tile's keys to their digit runs (SCATTER).  SCATTER ranks each key by
// one LDS atomic on the tile histogram, stages the tile in LDS in digit
// order and writes every run with consecutive lanes; when `perm` is given it
// also records, in input order, every key's slot in that staging order (its
// index among the tile's keys sorted by digit, below 2^16).
// 1024-thread workgroups are sized for two per CU (eight waves per SIMD, so
// at most 64 VGPRs), smaller ones for at least four waves per SIMD.
template <typename K, int THREADS, int ITEMS, int MAXD, int OP, int DIG>
__global__ __launch_bounds__(THREADS, THREADS >= 1024 ? 8 : 4) void k_msplit(const K* __restrict__ in, uint32_t n,
                                                    const SegPlan* __restrict__ plan, uint32_t nd, uint32_t log2P,
                                                    uint32_t P, const PartDesc* __restrict__ desc, uint32_t shift,
                                                    uint32_t* __restrict__ counts, K* __restrict__ out,
                                                    uint16_t* __restrict__ perm) {
  constexpr int TILE = THREADS * ITEMS;
  constexpr bool kCount = OP == OP_COUNT;
  constexpr int kDPT = (MAXD + THREADS - 1) / THREADS;  // digits per thread in the scan
  static_assert(TILE < 65536 && MAXD <= 65536, "digit and rank share a word");
  __shared__ uint32_t hist[MAXD];
  __shared__ uint32_t dstart[kCount ? 1 : MAXD];
  __shared__ uint32_t delta[kCount ? 1 : MAXD];  // output position of the digit's run minus dstart
  __shared__ uint32_t wtot[THREADS / kWave];
  __shared__ PartDesc sd[DIG == DIG_PART ? 1 : kMaxP];
  __shared__ uint32_t srange[DIG == DIG_RANGE ? kMaxP + 1 : 1];
  __shared__ K stage_k[kCount ? 1 : TILE];
  __shared__ uint16_t sdig[kCount ? 1 : TILE];

  const uint32_t t = threadIdx.x;
  TileLoc L;
  if (!tile_loc(plan, nd, n, TILE, L)) return;  // whole workgroup
  const uint32_t D = L.D, T = L.T, cb = L.cb, gs = L.gs, tl = L.tl, seg = L.seg;
  const uint32_t base = L.base, head = L.head, tail = L.tail;
  const uint32_t cnt = tail - head;  // keys of this tile
  const bool vec = head == 0 && tail == static_cast<uint32_t>(TILE) &&
                   (reinterpret_cast<uintptr_t>(in + base) & 15) == 0;

  // The tile's keys are requested first: they depend on nothing below, and
  // their round trip then overlaps the descriptor copy and the barrier.
  K v[ITEMS];
  uint32_t d[ITEMS];
  const uint32_t mask = load_items<K, THREADS, ITEMS>(in, base, head, tail, vec, v);

  if (DIG != DIG_PART) {
    // A batched table's segment brings its own descriptor (P == 1 there).
    const PartDesc* dsrc = (plan != nullptr && plan->desc_by_seg) ? desc + seg : desc;
    for (uint32_t i = t; i < P; i += THREADS) sd[i] = dsrc[i];
  }
  if (DIG == DIG_RANGE) {
    const uint32_t* bounds = reinterpret_cast<const uint32_t*>(desc + 1);
    for (uint32_t i = t; i <= D; i += THREADS) srange[i] = bounds[i];
  }
  for (uint32_t i = t; i < D; i += THREADS) hist[i] = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) in_regs(v[i]);
  __syncthreads();

  // Per-item values are computed for every item, valid or not (an invalid
  // item's key is 0, its digit in range); only memory effects are masked.
  // Conditional assignments to these arrays would make the compiler carry
  // them as whole vectors through every branch.
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (DIG == DIG_PART) {
      d[i] = part_of(KeyTraits<K>::hash(v[i]), log2P);
    } else if (DIG == DIG_RANGE) {
      // The last range starting at or below H (bounds[0] = 0, D <= 256).
      const uint32_t H = bucket_of(v[i], 0, sd);
      uint32_t lo = 0;
#pragma unroll
      for (uint32_t st = 128; st > 0; st >>= 1)
        if (lo + st < D && srange[lo + st] <= H) lo += st;
      d[i] = lo;
    } else {
      const uint32_t g = bucket_of(v[i], log2P, sd);
      d[i] = min((g - gs) >> shift, D - 1);
    }
  }

  // A wave whose first items mostly share one digit (a run of copies of
  // one key) groups its atomics; every other wave adds one per key.
  const bool skew = wave_skewed(d[0]);
  if (kCount) {
    if (skew) {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) lds_hist_add<false>(hist, d[i], (mask >> i) & 1u);
    } else if (vec) {
      // A whole tile (nearly every tile): no item is masked.
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) atomicAdd(&hist[d[i]], 1u);
    } else {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i)
        if ((mask >> i) & 1u) atomicAdd(&hist[d[i]], 1u);
    }
    __syncthreads();
    for (uint32_t dd = t; dd < D; dd += THREADS) counts[cb + dd * T + tl] = hist[dd];
    return;
  }

  // Rank of each key among the tile's keys of its digit (invalid items add 0).
  if (skew) {
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) d[i] |= lds_hist_add<true>(hist, d[i], (mask >> i) & 1u) << 16;
  } else {
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) d[i] |= atomicAdd(&hist[d[i]], (mask >> i) & 1u) << 16;
  }
  __syncthreads();

  // Digit starts in the tile (exclusive scan of the histogram; thread t
  // takes digits kDPT*t ..), and each run's output position.
  uint32_t c[kDPT], sum = 0;
#pragma unroll
  for (int x = 0; x < kDPT; ++x) {
    const uint32_t dd = kDPT * t + x;
    c[x] = dd < D ? hist[dd] : 0u;
    sum += c[x];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_sum<THREADS>(sum, wtot, total);
#pragma unroll
  for (int x = 0; x < kDPT; ++x) {
    const uint32_t dd = kDPT * t + x;
    if (dd < D) {
      dstart[dd] = ex;
      delta[dd] = counts[cb + dd * T + tl] - ex;
    }
    ex += c[x];
  }
  __syncthreads();

  // Stage the tile in digit order; d[i] becomes the key's staging slot.
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t dig = d[i] & 0xFFFFu;
    const uint32_t pos = dstart[dig] + (d[i] >> 16);
    if ((mask >> i) & 1u) {
      stage_k[pos] = v[i];
      sdig[pos] = static_cast<uint16_t>(dig);
    }
    d[i] = pos;
  }
  if (perm != nullptr) {
    constexpr int kVec = 16 / sizeof(K);
    if (vec) {
      // kVec consecutive keys per thread and load: one 8- or 4-byte store.
#pragma unroll
      for (int i = 0; i < ITEMS; i += kVec) {
        uint16_t* dst = perm + base + elem_of<K, THREADS>(true, i, t);
        if (kVec == 4)
          *reinterpret_cast<uint2*>(dst) = make_uint2(d[i] | (d[i + 1] << 16), d[i + 2] | (d[i + 3] << 16));
        else
          *reinterpret_cast<uint32_t*>(dst) = d[i] | (d[i + 1] << 16);
      }
    } else {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i)
        if ((mask >> i) & 1u) perm[base + elem_of<K, THREADS>(false, i, t)] = static_cast<uint16_t>(d[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t j = static_cast<uint32_t>(i) * THREADS + t;
    if (j < cnt) out[delta[sdig[j]] + j] = stage_k[j];
  }
}

// The inverse of a split applied to per-key counts, one split tile per
// workgroup, on the tiles of the split itself: the tile's digit runs of
// `src` (split order; run of digit d at the scanned count of (d, tile), its
// length up to the next entry) are copied into LDS in the tile's digit order,
// then out[i] = stage[perm[i]] for the tile's keys in input order: in the
// width they came in (OUT == GATHER_STAGE), as u32 (GATHER_COUNT), or as
// (stage[perm[i]] != 0) bytes (GATHER_FOUND).  The counts come as bytes when
// the table has no long bucket, else as u32.  Every global access reads or
// writes consecutive elements: a run, the slots, the output.
// SB: bytes per staged count.  Both widths are launched; the instance that
// does not match the table (bytes without long buckets) returns at once, so
// the byte instance, a quarter of the staging LDS, fits more workgroups.
template <int THREADS, int ITEMS, int MAXD, int OUT, int SB>
__global__ __launch_bounds__(THREADS, THREADS >= 1024 || (THREADS >= 512 && SB == 1) ? 8 : 4) void k_tile_gather(
    const uint16_t* __restrict__ perm, const void* __restrict__ src, uint32_t n,
    const SegPlan* __restrict__ plan, uint32_t nd, const uint32_t* __restrict__ scan,
    const uint32_t* __restrict__ unsorted, void* __restrict__ out) {
  constexpr int TILE = THREADS * ITEMS;
  constexpr int kDPT = (MAXD + THREADS - 1) / THREADS;
  constexpr int kW = THREADS / kWave;
  constexpr bool FOUND = OUT == GATHER_FOUND;
  static_assert(ITEMS % 4 == 0, "four slots per 8-byte load");
  static_assert(SB == 1 || SB == 4, "counts staged as bytes or words");
  using StageT = typename std::conditional<SB == 1, uint8_t, uint32_t>::type;
  __shared__ uint32_t dstart[MAXD + 1];
  __shared__ uint32_t delta[MAXD];  // src index of a slot minus the slot
  __shared__ uint32_t wtot[kW];
  __shared__ StageT stage[TILE];
  __shared__ __align__(16) uint16_t sdg[TILE];  // digit of each slot
  const uint32_t t = threadIdx.x;
  // Counts as bytes in src, and in out for a further gather.  A scalar load:
  // the instance that does not serve this table has every workgroup read the
  // flag and leave, so that read's latency is all it costs.
  const bool narrow = ld_uniform(unsorted, kHasLongWord) == 0;
  if (narrow != (SB == 1)) return;  // the other instance serves this table
  TileLoc L;
  if (!tile_loc(plan, nd, n, TILE, L)) return;  // whole workgroup
  const uint32_t cnt = L.tail - L.head;         // at least 1: a tile holds keys
  const uint32_t first = L.base + L.head;       // input order: elements first + e, e < cnt
  const bool out_bytes = FOUND || (OUT == GATHER_STAGE && narrow);
  const uintptr_t oa = out_bytes ? reinterpret_cast<uintptr_t>(static_cast<uint8_t*>(out) + first)
                                 : reinterpret_cast<uintptr_t>(static_cast<uint32_t*>(out) + first);
  const bool vec = cnt == static_cast<uint32_t>(TILE) && (first & 3u) == 0 &&
                   (reinterpret_cast<uintptr_t>(perm + first) & 7u) == 0 && (oa & (out_bytes ? 3u : 15u)) == 0;

  // The slots of the tile's keys (input order) are needed last but depend on
  // nothing: they are requested first, four per thread and load.
  uint2 pv[ITEMS / 4];
  if (vec) {
#pragma unroll
    for (int r = 0; r < ITEMS / 4; ++r)
      pv[r] = *reinterpret_cast<const uint2*>(perm + first + static_cast<uint32_t>(r) * (THREADS * 4) + 4 * t);
  }

  // Runs of the tile's digits: start in src and length (the entry after
  // (d, tile) is (d, tile + 1), or (d + 1, 0); after the segment's last entry
  // comes the segment's end).
  uint32_t c[kDPT], s0[kDPT], sum = 0;
#pragma unroll
  for (int x = 0; x < kDPT; ++x) {
    const uint32_t dd = kDPT * t + x;
    c[x] = 0;
    s0[x] = 0;
    if (dd < L.D) {
      const uint32_t at = L.cb + dd * L.T + L.tl;
      s0[x] = scan[at];
      c[x] = (dd + 1 == L.D && L.tl + 1 == L.T ? L.k1 : scan[at + 1]) - s0[x];
    }
    sum += c[x];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_sum<THREADS>(sum, wtot, total);
#pragma unroll
  for (int x = 0; x < kDPT; ++x) {
    const uint32_t dd = kDPT * t + x;
    if (dd < L.D) {
      dstart[dd] = ex;
      delta[dd] = s0[x] - ex;
    }
    ex += c[x];
  }
  if (t == 0) dstart[L.D] = total;
  __syncthreads();

  // Digit of every slot.  Thread t takes slots ITEMS t .. ITEMS t + ITEMS - 1:
  // a binary search over the run starts finds the digit of the first (an
  // empty run shares its successor's start, so the last digit whose start
  // is at or below the slot holds it; dstart[0] = 0 and dstart[D] = cnt
  // bound the search), then a walk over the consecutive slots.  Every
  // thread's search runs at once, where marking run by run took one
  // dependent LDS round trip per digit and wave.
  {
    static_assert(ITEMS % 8 == 0, "whole 16-byte stores of slot digits");
    const uint32_t j0 = static_cast<uint32_t>(ITEMS) * t;
    if (j0 < cnt) {
      uint32_t lo = 0, hi = L.D;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (dstart[mid] <= j0)
          lo = mid;
        else
          hi = mid;
      }
      uint32_t d = lo, dg[ITEMS / 2];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = j0 + static_cast<uint32_t>(i);
        while (d + 1 < L.D && dstart[d + 1] <= j) ++d;  // stops at the run holding j (j < cnt = dstart[D])
        if (i & 1) dg[i >> 1] |= d << 16; else dg[i >> 1] = d;
      }
      if (j0 + ITEMS <= cnt) {
        uint4* dst = reinterpret_cast<uint4*>(sdg + j0);
#pragma unroll
        for (int x = 0; x < ITEMS / 8; ++x) dst[x] = make_uint4(dg[4 * x], dg[4 * x + 1], dg[4 * x + 2], dg[4 * x + 3]);
      } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
          if (j0 + i < cnt) sdg[j0 + i] = static_cast<uint16_t>(dg[i >> 1] >> ((i & 1) << 4));
      }
    }
  }
  __syncthreads();

  // Slot j takes src[delta[digit] + j]: consecutive slots of a run read
  // consecutive elements.  Lanes past the tile's end redo its last slot and
  // store nothing.
  uint32_t v[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t j = min(static_cast<uint32_t>(i) * THREADS + t, cnt - 1);
    v[i] = delta[sdg[j]] + j;
  }
  if (narrow) {
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) v[i] = static_cast<const uint8_t*>(src)[v[i]];
  } else {
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) v[i] = static_cast<const uint32_t*>(src)[v[i]];
  }
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t j = static_cast<uint32_t>(i) * THREADS + t;
    if (j < cnt) stage[j] = static_cast<StageT>(v[i]);
  }
  __syncthreads();

  if (vec) {
    // Four consecutive elements per thread and round.
#pragma unroll
    for (int r = 0; r < ITEMS / 4; ++r) {
      const uint32_t e = first + static_cast<uint32_t>(r) * (THREADS * 4) + 4 * t;
      const uint32_t a = stage[pv[r].x & 0xFFFFu], b = stage[pv[r].x >> 16], cc = stage[pv[r].y & 0xFFFFu],
                     dd = stage[pv[r].y >> 16];
      if (FOUND)
        *reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(out) + e) =
            (a != 0 ? 1u : 0u) | (b != 0 ? 0x100u : 0u) | (cc != 0 ? 0x10000u : 0u) | (dd != 0 ? 0x1000000u : 0u);
      else if (out_bytes)  // byte counts below 256
        *reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(out) + e) = a | (b << 8) | (cc << 16) | (dd << 24);
      else
        *reinterpret_cast<uint4*>(static_cast<uint32_t*>(out) + e) = make_uint4(a, b, cc, dd);
    }
    return;
  }
  for (uint32_t e = t; e < cnt; e += THREADS) {
    const uint32_t x = stage[perm[first + e]];
    if (FOUND)
      static_cast<uint8_t*>(out)[first + e] = x != 0 ? 1 : 0;
    else if (out_bytes)
      static_cast<uint8_t*>(out)[first + e] = static_cast<uint8_t>(x);
    else
      static_cast<uint32_t*>(out)[first + e] = x;
  }
}

// ------------------------------------------------------------------ plan
constexpr int kPlanThreads = 1024;

// One workgroup walks the segments in chunks of kPlanThreads, carrying the
// three running prefix sums (tiles, counts, sub-bins) across chunks.
__global__ __launch_bounds__(kPlanThreads) void k_plan(const uint32_t* __restrict__ scan1, uint32_t tiles1,
                                                       uint32_t nseg, uint32_t n, int mode,
                                                       const uint32_t* __restrict__ bb,
                                                       const uint32_t* __restrict__ nb_total,
                                                       const uint32_t* __restrict__ seg_keys, uint32_t sh1,
                                                       uint32_t log2S, uint32_t tile2, uint32_t max_tiles,
                                                       uint32_t max_subbins, uint32_t* __restrict__ offsets,
                                                       SegPlan* __restrict__ plan) {
  __shared__ uint32_t wtot[kPlanThreads / kWave];
  const uint32_t t = threadIdx.x;
  const uint32_t NB = *nb_total;
  uint32_t* arr = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(plan) + (sizeof(SegPlan) + 255) / 256 * 256);
  const size_t stride = static_cast<size_t>(nseg) + 1;
  uint32_t* key0a = arr;
  uint32_t* g0a = arr + stride;
  uint32_t* Da = arr + 2 * stride;
  uint32_t* Ta = arr + 3 * stride;
  uint32_t* tfa = arr + 4 * stride;
  uint32_t* cba = arr + 5 * stride;
  uint32_t* sba = arr + 6 * stride;
  auto key_start = [&](uint32_t x) -> uint32_t {
    if (x >= nseg) return n;
    if (mode == 2) return seg_keys[x];
    return tiles1 != 0 ? scan1[static_cast<size_t>(x) * tiles1] : 0u;
  };
  auto bucket_start = [&](uint32_t x) -> uint32_t {
    if (x >= nseg) return NB;
    if (mode == 1) return static_cast<uint32_t>(min(static_cast<uint64_t>(x) << sh1, static_cast<uint64_t>(NB)));
    return bb[x];
  };
  uint32_t cT = 0, cC = 0, cD = 0;
  for (uint32_t c0 = 0; c0 < nseg; c0 += kPlanThreads) {
    const uint32_t x = c0 + t;
    uint32_t key0 = 0, g0 = 0, T = 0, D = 0;
    if (x < nseg) {
      key0 = key_start(x);
      g0 = bucket_start(x);
      const uint32_t key1 = key_start(x + 1), g1 = bucket_start(x + 1);
      T = key1 > key0 ? (key1 - (key0 & ~(kTileAlign - 1)) + tile2 - 1) / tile2 : 0u;
      const uint64_t R = g1 - g0;
      D = R == 0 ? 0u
                 : static_cast<uint32_t>(min((R + (1ull << log2S) - 1) >> log2S, static_cast<uint64_t>(kMaxD2)));
    }
    uint32_t sT, sC, sD;
    const uint32_t tf = block_exclusive_sum<kPlanThreads>(T, wtot, sT);
    const uint32_t cbv = block_exclusive_sum<kPlanThreads>(D * T, wtot, sC);
    const uint32_t sbf = block_exclusive_sum<kPlanThreads>(D, wtot, sD);
    if (x < nseg) {
      key0a[x] = key0;
      g0a[x] = g0;
      Da[x] = D;
      Ta[x] = T;
      tfa[x] = cT + tf;
      cba[x] = cC + cbv;
      sba[x] = cD + sbf;
    }
    cT += sT;
    cC += sC;
    cD += sD;
  }
  if (t == 0) {
    key0a[nseg] = n;
    g0a[nseg] = NB;
    Da[nseg] = 0;
    Ta[nseg] = 0;
    tfa[nseg] = cT;
    cba[nseg] = cC;
    sba[nseg] = cD;
    plan->nseg = nseg;
    plan->total_tiles = cT;
    plan->total_counts = cC;
    plan->total_subbins = cD;
    plan->num_buckets = NB;
    plan->n = n;
    plan->tile_keys = tile2;
    plan->log2S = log2S;
    plan->desc_by_seg = mode == 2 ? 1u : 0u;
    plan->max_tiles = max_tiles;
    plan->max_subbins = max_subbins;
    plan->pad = 0;
    plan->tile_seg = arr + kPlanArrays * stride;
    plan->sb_seg = arr + kPlanArrays * stride + max_tiles;
    plan->key0 = key0a;
    plan->g0 = g0a;
    plan->D = Da;
    plan->T = Ta;
    plan->tile_first = tfa;
    plan->cbase = cba;
    plan->sb_first = sba;
    if (offsets != nullptr) offsets[NB] = n;
  }
}

// tile_seg / sb_seg: the segment of every level-2 tile and sub-bin (one
// binary search per entry, all in parallel, instead of one per workgroup in
// every later pass).  Entries past the totals are left unwritten.
__global__ __launch_bounds__(256) void k_seg_map(const SegPlan* __restrict__ plan) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  const uint32_t nt = plan->total_tiles, ns = plan->total_subbins;
  if (i < nt) plan->tile_seg[i] = find_segment(plan->tile_first, plan->nseg, i);
  if (i < ns) plan->sb_seg[i] = find_segment(plan->sb_first, plan->nseg, i);
}

// Layout of a batch of tables (see launch_batch_layout).  Thread t owns the
// contiguous entries [x0, x1) of the offsets 0..T and walks them three times:
// (1) the largest clamped offset, then a max-scan over the threads in LDS;
// (2) the sum of its tables' sizes V_x, then an exclusive sum over the
// threads; (3) the clamped offsets, bucket bases and descriptors.  With
// bb == nullptr only the clamped offsets are written.
__global__ __launch_bounds__(kPlanThreads) void k_batch_layout(const uint32_t* __restrict__ tk, uint32_t T,
                                                               uint32_t n, uint32_t num, uint32_t den,
                                                               uint32_t* __restrict__ po, uint32_t* __restrict__ bb,
                                                               PartDesc* __restrict__ desc) {
  __shared__ uint32_t smax[kPlanThreads];
  __shared__ uint32_t wtot[kPlanThreads / kWave];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (T + 1 + kPlanThreads - 1) / kPlanThreads;
  const uint32_t x0 = min(T + 1, t * per), x1 = min(T + 1, x0 + per);
  // Entry x clamped: 0 at x = 0, n at x = T, otherwise at most n.
  auto val = [&](uint32_t x) -> uint32_t { return x == 0 ? 0u : (x == T ? n : min(tk[x], n)); };
  uint32_t m = 0;
  for (uint32_t x = x0; x < x1; ++x) m = max(m, val(x));
  smax[t] = m;
  __syncthreads();
  for (uint32_t off = 1; off < kPlanThreads; off <<= 1) {
    const uint32_t o = t >= off ? smax[t - off] : 0u;
    __syncthreads();
    smax[t] = max(smax[t], o);
    __syncthreads();
  }
  const uint32_t before = t == 0 ? 0u : smax[t - 1];
  const uint32_t xe = min(x1, T);  // tables owned: [x0, xe)
  auto size_of = [&](uint32_t nt) -> uint32_t {
    const uint64_t v = static_cast<uint64_t>(nt) * num / den;
    return static_cast<uint32_t>(v < 1 ? 1 : v);
  };
  uint32_t sumV = 0;
  if (bb != nullptr && x0 < xe) {
    uint32_t cur = max(before, val(x0));
    for (uint32_t x = x0; x < xe; ++x) {
      const uint32_t nxt = max(cur, val(x + 1));
      sumV += size_of(nxt - cur);
      cur = nxt;
    }
  }
  uint32_t total = 0;
  uint32_t base = bb != nullptr ? block_exclusive_sum<kPlanThreads>(sumV, wtot, total) : 0u;
  uint32_t cur = x0 < x1 ? max(before, val(x0)) : 0u;
  for (uint32_t x = x0; x < x1; ++x) {
    po[x] = cur;
    if (bb != nullptr && x < T) {
      const uint32_t nxt = max(cur, val(x + 1));
      const uint32_t V = size_of(nxt - cur);
      desc[x] = make_desc(V, base);
      bb[x] = base;
      base += V;
      cur = nxt;
    } else if (x < T) {
      cur = max(cur, val(x + 1));
    }
  }
  if (bb != nullptr && t == 0) bb[T] = total;
}

// Sub-bin `b` of a plan: its segment, bucket range [gA, gB) and key range
// [kA, kB) in the level-2 output (scan2 = scanned level-2 counts).
struct SubBin {
  uint32_t gA, gB, kA, kB, seg;
};

// kScalar: read the plan through scalar loads (ld_uniform).  Measured at
// 2^28 keys: the probe gains (0.85 -> 0.81 ms), the LDS build loses (0.55
// -> 0.65 ms; its waits on LDS operations also wait on scalar loads, and it
// is bound by instruction issue), so the build keeps vector loads.
template <bool kScalar>
__device__ __forceinline__ SubBin sub_bin(const SegPlan* plan, const uint32_t* scan2, uint32_t b) {
  auto at = [](const uint32_t* p, uint32_t i) { return kScalar ? ld_uniform(p, i) : p[i]; };
  const uint32_t seg = at(plan->sb_seg, b);
  const uint32_t d = b - at(plan->sb_first, seg);
  const uint32_t D = at(plan->D, seg), T = at(plan->T, seg);
  SubBin s;
  s.gA = at(plan->g0, seg) + (d << plan->log2S);
  s.gB = (d + 1 == D) ? at(plan->g0, seg + 1) : s.gA + (1u << plan->log2S);
  s.kA = T != 0 ? at(scan2, at(plan->cbase, seg) + d * T) : at(plan->key0, seg);
  s.kB = (d + 1 < D) ? (T != 0 ? at(scan2, at(plan->cbase, seg) + (d + 1) * T) : at(plan->key0, seg))
                     : at(plan->key0, seg + 1);
  s.seg = seg;
  return s;
}

// ------------------------------------------------------------- LDS build
// A sub-bin of m <= 65535 keys is sorted in LDS: with one 32-bit counter per
// bucket when R <= kWideR (the common sub-bin), else with 16-bit counters,
// two per word (bucket i in half i & 1 of word i >> 1), up to R <= kSMax.
// The same LDS then stages the sorted keys so that they leave in whole lines.
constexpr uint32_t kBuildWords = 8448;  // 33 KiB: the counters, then the staging area (four
                                        // workgroups per CU with the descriptors)
constexpr uint32_t kSMax = 1u << 14;     // 16-bit counters for up to this many buckets
constexpr uint32_t kWideR = 8192;        // 32-bit counters for up to this many buckets
constexpr uint32_t kHeavyChunk = kBuildThreads * 20;  // keys per workgroup of the heavy passes
static_assert(kSMax <= 2 * kBuildWords, "16-bit counters fit the LDS block");
static_assert(kWideR <= kBuildWords, "32-bit counters fit the LDS block");

// Exclusive scan in place of the R 16-bit counters packed in c[0 .. (R+1)/2).
// Each wave scans one contiguous chunk of words in rounds of 64, then adds the
// totals of the chunks before it.  Every prefix fits 16 bits (m <= 65535).
template <int THREADS>
__device__ __forceinline__ void lds_exclusive_scan16(uint32_t* c, uint32_t R, uint32_t* wsum) {
  constexpr int W = THREADS / kWave;
  const uint32_t words = (R + 1) >> 1;
  const uint32_t ch = ((words + W - 1) / W + kWave - 1) / kWave * kWave;
  const uint32_t w = threadIdx.x / kWave, l = lane_id();
  uint32_t carry = 0;
  for (uint32_t r0 = 0; r0 < ch; r0 += kWave) {
    const uint32_t idx = w * ch + r0 + l;
    const uint32_t x = idx < words ? c[idx] : 0u;
    const uint32_t lo = x & 0xFFFFu, sum = lo + (x >> 16);
    const uint32_t inc = wave_inclusive_sum(sum);
    const uint32_t ex = carry + inc - sum;
    if (idx < words) c[idx] = ex | ((ex + lo) << 16);
    carry += readlane(inc, kWave - 1);
  }
  if (l == 0) wsum[w] = carry;
  __syncthreads();
  uint32_t base = 0;
#pragma unroll
  for (int x = 0; x < W; ++x) base += (x < static_cast<int>(w)) ? wsum[x] : 0u;
  const uint32_t add = base | (base << 16);
  for (uint32_t r0 = 0; r0 < ch; r0 += kWave) {
    const uint32_t idx = w * ch + r0 + l;
    if (idx < words) c[idx] += add;
  }
  __syncthreads();
}

// Exclusive scan in place of R 32-bit counters c[0 .. R): each wave scans
// one contiguous chunk in rounds of 64, then adds the totals of the chunks
// before it.
template <int THREADS>
__device__ __forceinline__ void lds_exclusive_scan32(uint32_t* c, uint32_t R, uint32_t* wsum) {
  constexpr int W = THREADS / kWave;
  const uint32_t ch = ((R + W - 1) / W + kWave - 1) / kWave * kWave;
  const uint32_t w = threadIdx.x / kWave, l = lane_id();
  uint32_t carry = 0;
  for (uint32_t r0 = 0; r0 < ch; r0 += kWave) {
    const uint32_t idx = w * ch + r0 + l;
    const uint32_t x = idx < R ? c[idx] : 0u;
    const uint32_t inc = wave_inclusive_sum(x);
    if (idx < R) c[idx] = carry + inc - x;
    carry += readlane(inc, kWave - 1);
  }
  if (l == 0) wsum[w] = carry;
  __syncthreads();
  uint32_t base = 0;
#pragma unroll
  for (int x = 0; x < W; ++x) base += (x < static_cast<int>(w)) ? wsum[x] : 0u;
  for (uint32_t r0 = 0; r0 < ch; r0 += kWave) {
    const uint32_t idx = w * ch + r0 + l;
    if (idx < R) c[idx] += base;
  }
  __syncthreads();
}

// LDS counter add for every valid lane; the lanes whose index equals the
// first valid lane's share one atomic (a bucket holding one heavy key then
// costs one atomic per wave).  With kReturn, each lane gets a distinct old
// value (its position).
template <bool kReturn, bool kPacked = false>
__device__ __forceinline__ uint32_t lds_agg_add(uint32_t* ctr, uint32_t idx, bool valid) {
  // kPacked: counter idx is the 16-bit half idx & 1 of word idx >> 1.
  const uint64_t act = ballot(valid);
  if (act == 0) return 0;
  const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(act)) - 1);
  const uint32_t li = readlane(idx, leader);
  const bool in = valid && idx == li;
  const uint64_t same = ballot(in);
  const uint32_t sh = kPacked ? (idx & 1u) << 4 : 0u;
  const uint32_t w = kPacked ? idx >> 1 : idx;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(&ctr[w], popc64(same) << sh);
  uint32_t pos = 0;
  if (kReturn) {
    base = readlane(base, leader);
    if (in) pos = (kPacked ? (base >> sh) & 0xFFFFu : base) + popc64(same & lanemask_lt());
    else if (valid) pos = kPacked ? (atomicAdd(&ctr[w], 1u << sh) >> sh) & 0xFFFFu : atomicAdd(&ctr[w], 1u);
  } else if (valid && !in) {
    atomicAdd(&ctr[w], 1u << sh);
  }
  return pos;
}

__device__ __forceinline__ uint32_t ld_l2(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_l2(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Appends long bucket g (len keys) to its list.  Both lists share one
// array of ctr[4] entries: buckets of at most kWaveLong keys from the front
// (ctr[0] of them), longer ones from the back (ctr[2]).
__device__ __forceinline__ void note_long(uint32_t* ctr, uint32_t* list, uint32_t g, uint32_t len) {
  if (len <= kWaveLong)
    list[atomicAdd(&ctr[0], 1u)] = g;
  else
    list[ctr[4] - 1 - atomicAdd(&ctr[2], 1u)] = g;
}

// The keys of one sub-bin, each with its position p < m packed as 16-bit
// halves of pos (key j in half j & 1 of word j >> 1), staged in LDS in
// position order and written to out[0 .. m) in whole lines, in chunks of
// what the LDS block holds.  Every thread of the workgroup calls it; the LDS
// block is free on entry (after a barrier).
template <typename K, int THREADS, int REG>
__device__ __forceinline__ void stage_out(uint32_t* lds, const uint32_t* pos, const K* v, uint32_t m,
                                          K* __restrict__ out) {
  constexpr uint32_t kStageKeys = kBuildWords * 4 / sizeof(K);
  const uint32_t t = threadIdx.x;
  K* stage = reinterpret_cast<K*>(lds);
  if (m <= kStageKeys) {
    // One chunk (the usual case): no range test per key.
#pragma unroll
    for (int j = 0; j < REG; ++j) {
      const uint32_t e = static_cast<uint32_t>(j) * THREADS + t;
      if (e < m) stage[(pos[j >> 1] >> ((j & 1) << 4)) & 0xFFFFu] = v[j];
    }
    __syncthreads();
    for (uint32_t i = t; i < m; i += THREADS) out[i] = stage[i];
    return;
  }
  for (uint32_t h0 = 0; h0 < m; h0 += kStageKeys) {
#pragma unroll
    for (int j = 0; j < REG; ++j) {
      const uint32_t e = static_cast<uint32_t>(j) * THREADS + t;
      const uint32_t p = (pos[j >> 1] >> ((j & 1) << 4)) & 0xFFFFu;
      if (e < m && p >= h0 && p < h0 + kStageKeys) stage[p - h0] = v[j];
    }
    __syncthreads();
    const uint32_t len = min(kStageKeys, m - h0);
    for (uint32_t i = t; i < len; i += THREADS) out[h0 + i] = stage[i];
    __syncthreads();
  }
}

// f(key, e) for each e < m of thread t's stride (t, t + THREADS, ...), with
// U loads in flight per thread: a lane past the end re-reads the last key
// and skips the call.  m > 0.
template <int THREADS, int U, typename K, typename F>
__device__ __forceinline__ void for_keys(const K* __restrict__ a, uint32_t m, uint32_t t, F&& f) {
  for (uint32_t e0 = 0; e0 < m; e0 += THREADS * U) {
    K x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = a[min(e0 + static_cast<uint32_t>(u) * THREADS + t, m - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t e = e0 + static_cast<uint32_t>(u) * THREADS + t;
      if (e < m) f(x[u], e);
    }
  }
}

// MINW: waves per SIMD to fit (8: two workgroups of 1024 threads per CU).
template <typename K, int THREADS, int REG, int MINW>
__global__ __launch_bounds__(THREADS, MINW) void k_lds_build(const K* __restrict__ in,
                                                             const SegPlan* __restrict__ plan,
                                                             const uint32_t* __restrict__ scan2, uint32_t log2P,
                                                             uint32_t P, const PartDesc* __restrict__ desc,
                                                             uint32_t* __restrict__ offsets, K* __restrict__ out,
                                                             uint32_t* __restrict__ long_count,
                                                             uint32_t* __restrict__ long_list,
                                                             uint32_t* __restrict__ heavy_count,
                                                             uint32_t* __restrict__ heavy_chunks,
                                                             uint32_t* __restrict__ heavy_bins,
                                                             uint32_t* __restrict__ long_flags) {
  __shared__ uint32_t lds[kBuildWords];
  __shared__ PartDesc sd[kMaxP];
  __shared__ uint32_t wsum[THREADS / kWave];
  __shared__ uint32_t lbase[2];  // this sub-bin's first entries in the long-bucket list, front and back
  constexpr int kFlight = 8;  // loads in flight per thread in the loops over oversized sub-bins
  const uint32_t t = threadIdx.x;
  if (blockIdx.x >= plan->total_subbins) return;  // whole workgroup
  const SubBin sb = sub_bin<false>(plan, scan2, blockIdx.x);
  const uint32_t R = sb.gB - sb.gA, m = sb.kB - sb.kA;
  {
    const PartDesc* dsrc = plan->desc_by_seg ? desc + sb.seg : desc;
    for (uint32_t i = t; i < P; i += THREADS) sd[i] = dsrc[i];
  }

  if (R <= kWideR && m <= 0xFFFFu) {
    // The common sub-bin (at most 2^13 buckets): one 32-bit counter per
    // bucket, so no key pays for packing.  Thread t scans its CPT counters
    // CPT t .. CPT t + CPT - 1 in registers, which also shows it the long
    // buckets; the offsets then leave in one coalesced pass.
    constexpr int CPT = static_cast<int>(kWideR) / THREADS, CQ = CPT / 4;
    static_assert(CPT * THREADS == static_cast<int>(kWideR) && CPT % 4 == 0 && CPT <= 16,
                  "whole uint4 groups of at most sixteen counters per thread");
    uint4* lds4 = reinterpret_cast<uint4*>(lds);
    for (uint32_t i = t; i < kWideR / 4; i += THREADS) lds4[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    // Counters to exclusive offsets, in LDS (the scatter's cursors) and out.
    auto scan_counters = [&]() {
      uint32_t c[CPT];
#pragma unroll
      for (int x = 0; x < CQ; ++x) {
        const uint4 q = lds4[CQ * t + x];
        c[4 * x] = q.x;
        c[4 * x + 1] = q.y;
        c[4 * x + 2] = q.z;
        c[4 * x + 3] = q.w;
      }
      uint32_t sum = 0;
#pragma unroll
      for (int k = 0; k < CPT; ++k) sum += c[k];
      if constexpr (sizeof(K) == 4) {
        // 32-bit keys: the register path holds this kernel at 64 VGPRs
        // (eight waves per SIMD), and every variant of the reservation below
        // spilled here; a sub-bin with long buckets is only flagged, and
        // k_note_long lists them from the bucket starts written below.
        uint32_t total;
        uint32_t ex = block_exclusive_sum<THREADS>(sum, wsum, total);
#pragma unroll
        for (int x = 0; x < CQ; ++x) {
          uint4 q;
          q.x = ex;
          q.y = q.x + c[4 * x];
          q.z = q.y + c[4 * x + 1];
          q.w = q.z + c[4 * x + 2];
          ex = q.w + c[4 * x + 3];
          lds4[CQ * t + x] = q;
        }
        uint32_t mx = 0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) mx = max(mx, c[k]);
        if (ballot(mx > kLongT) != 0 && lane_id() == 0) long_flags[blockIdx.x] = 1u;  // same value from any wave
        __syncthreads();
      } else {
        // One scan carries three sums: keys (bits 0-15, at most
        // m <= 65535), long buckets for the front of the long-bucket list
        // (bits 16-25) and for its back (bits 26-31); a long bucket has more
        // than kLongT keys, so there are at most 1008 of them.  The
        // workgroup then reserves its entries with one atomic per end
        // instead of one per bucket: atomics on one address are served one
        // at a time, and a skewed table has long buckets in almost every
        // sub-bin.  Bit k of marks: bucket CPT t + k is long; bit 16 + k: it
        // goes to the back (more than kWaveLong keys).
        uint32_t marks = 0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          marks |= (c[k] > kLongT ? 1u : 0u) << k;
          marks |= (c[k] > kWaveLong ? 1u : 0u) << (16 + k);
        }
        const uint32_t nback = __popc(marks >> 16), nfront = __popc(marks & 0xFFFFu) - nback;
        uint32_t total;
        const uint32_t exs = block_exclusive_sum<THREADS>(sum | (nfront << 16) | (nback << 26), wsum, total);
        uint32_t ex = exs & 0xFFFFu;
#pragma unroll
        for (int x = 0; x < CQ; ++x) {
          uint4 q;
          q.x = ex;
          q.y = q.x + c[4 * x];
          q.z = q.y + c[4 * x + 1];
          q.w = q.z + c[4 * x + 2];
          ex = q.w + c[4 * x + 3];
          lds4[CQ * t + x] = q;
        }
        const uint32_t tfront = (total >> 16) & 0x3FFu, tback = total >> 26;
        if (t == 0) {
          if (tfront != 0) lbase[0] = atomicAdd(&long_count[0], tfront);
          if (tback != 0) lbase[1] = atomicAdd(&long_count[2], tback);
        }
        __syncthreads();
        if (marks != 0) {
          uint32_t f = lbase[0] + ((exs >> 16) & 0x3FFu), b = lbase[1] + (exs >> 26);
          for (uint32_t left = marks & 0xFFFFu; left != 0; left &= left - 1) {
            const uint32_t k = static_cast<uint32_t>(__ffs(left)) - 1;
            const uint32_t g = sb.gA + CPT * t + k;
            if ((marks >> (16 + k)) & 1u)
              long_list[long_count[4] - 1 - b++] = g;
            else
              long_list[f++] = g;
          }
        }
      }
      for (uint32_t i = t; i < R; i += THREADS) offsets[sb.gA + i] = sb.kA + lds[i];
      __syncthreads();
    };
    if (m > static_cast<uint32_t>(THREADS * REG)) {
      // More keys than the registers hold: two passes over them in global
      // memory, positions straight to global memory.  A branch of its own,
      // so that nothing of it stays live across the register path's scan.
      for_keys<THREADS, kFlight>(in + sb.kA, m, t,
                                 [&](K key, uint32_t) { lds_agg_add<false>(lds, bucket_of(key, log2P, sd) - sb.gA, true); });
      __syncthreads();
      scan_counters();
      for_keys<THREADS, kFlight>(in + sb.kA, m, t, [&](K key, uint32_t) {
        out[sb.kA + lds_agg_add<true>(lds, bucket_of(key, log2P, sd) - sb.gA, true)] = key;
      });
      return;
    }
    K v[REG];
    uint32_t pos[(REG + 1) / 2];  // two 16-bit values per word: bucket, then position
    if (m > 0) {
      const uint32_t last = m - 1;
#pragma unroll
      for (int j = 0; j < REG; ++j) v[j] = in[sb.kA + min(static_cast<uint32_t>(j) * THREADS + t, last)];
#pragma unroll
      for (int j = 0; j < REG; ++j) {
        const uint32_t e = static_cast<uint32_t>(j) * THREADS + t;
        const uint32_t lb = bucket_of(v[j], log2P, sd) - sb.gA;
        if (e < m) atomicAdd(&lds[lb], 1u);
        if (j & 1) pos[j >> 1] |= lb << 16; else pos[j >> 1] = lb;
      }
    }
    __syncthreads();
    scan_counters();
#pragma unroll
    for (int j = 0; j < REG; ++j) {
      const uint32_t e = static_cast<uint32_t>(j) * THREADS + t;
      const uint32_t lb = (pos[j >> 1] >> ((j & 1) << 4)) & 0xFFFFu;
      uint32_t p = 0;
      if (e < m) p = atomicAdd(&lds[lb], 1u);
      pos[j >> 1] = (pos[j >> 1] & ~(0xFFFFu << ((j & 1) << 4))) | (p << ((j & 1) << 4));
    }
    __syncthreads();  // every position is known: the counters are dead
    stage_out<K, THREADS, REG>(lds, pos, v, m, out + sb.kA);
    return;
  }

  if (R <= kSMax && m <= 0xFFFFu) {
    for (uint32_t i = t; i < (R + 1) / 2; i += THREADS) lds[i] = 0;
    __syncthreads();
    const bool regs = m <= static_cast<uint32_t>(THREADS * REG);
    K v[REG];
    // Two 16-bit values per word: first each key's bucket in the sub-bin
    // (R <= kSMax), then its position (m <= 65535).
    uint32_t pos[(REG + 1) / 2];
    if (regs && m > 0) {
      // Every load first, all in flight at once: a lane past the sub-bin's
      // end re-reads its last key (its counter add is skipped), so nothing
      // between the loads depends on a branch.
      const uint32_t last = m - 1;
#pragma unroll
      for (int j = 0; j < REG; ++j) v[j] = in[sb.kA + min(static_cast<uint32_t>(j) * THREADS + t, last)];
#pragma unroll
      for (int j = 0; j < REG; ++j) {
        const uint32_t e = static_cast<uint32_t>(j) * THREADS + t;
        const uint32_t lb = bucket_of(v[j], log2P, sd) - sb.gA;
        if (e < m) atomicAdd(&lds[lb >> 1], 1u << ((lb & 1u) << 4));
        if (j & 1) pos[j >> 1] |= lb << 16; else pos[j >> 1] = lb;
      }
    } else if (!regs) {
      for_keys<THREADS, kFlight>(in + sb.kA, m, t,
                                 [&](K key, uint32_t) { lds_agg_add<false, true>(lds, bucket_of(key, log2P, sd) - sb.gA, true); });
    }
    __syncthreads();
    lds_exclusive_scan16<THREADS>(lds, R, wsum);
    for (uint32_t i = t; i < R; i += THREADS) {
      const uint32_t e0 = get_half(lds, i);
      offsets[sb.gA + i] = sb.kA + e0;
      const uint32_t e1 = i + 1 < R ? get_half(lds, i + 1) : m;
      if (e1 - e0 > kLongT) note_long(long_count, long_list, sb.gA + i, e1 - e0);
    }
    __syncthreads();
    if (!regs) {
      // Oversized sub-bin: positions go straight to global memory.
      for_keys<THREADS, kFlight>(in + sb.kA, m, t, [&](K key, uint32_t) {
        out[sb.kA + lds_agg_add<true, true>(lds, bucket_of(key, log2P, sd) - sb.gA, true)] = key;
      });
      return;
    }
#pragma unroll
    for (int j = 0; j < REG; ++j) {
      const uint32_t e = static_cast<uint32_t>(j) * THREADS + t;
      const uint32_t lb = (pos[j >> 1] >> ((j & 1) << 4)) & 0xFFFFu, sh = (lb & 1u) << 4;
      uint32_t p = 0;
      if (e < m) p = (atomicAdd(&lds[lb >> 1], 1u << sh) >> sh) & 0xFFFFu;
      pos[j >> 1] = (pos[j >> 1] & ~(0xFFFFu << ((j & 1) << 4))) | (p << ((j & 1) << 4));
    }
    __syncthreads();  // every position is known: the counters are dead
    stage_out<K, THREADS, REG>(lds, pos, v, m, out + sb.kA);
    return;
  }

  if (R <= kWideR) {
    // More than 65535 keys (heavy keys): the sub-bin is shared by the
    // workgroups of the heavy passes below.  Here its counters (its own
    // offsets) start at zero and its chunks are queued.
    for (uint32_t i = t; i < R; i += THREADS) offsets[sb.gA + i] = 0u;
    if (t == 0) {
      const uint32_t nch = (m + kHeavyChunk - 1) / kHeavyChunk;
      const uint32_t at = atomicAdd(&heavy_count[0], nch);
      for (uint32_t k = 0; k < nch; ++k) {
        heavy_chunks[2 * (at + k)] = blockIdx.x;
        heavy_chunks[2 * (at + k) + 1] = k;
      }
      heavy_bins[atomicAdd(&heavy_count[1], 1u)] = blockIdx.x;
    }
    return;
  }

  // A sub-bin wider than LDS (a level-1 segment with more buckets than its
  // sub-bins can hold folds its tail into the last one): the same three
  // steps with the counters in global memory, offsets[gA + i] serving as the
  // counter of bucket i.
  __syncthreads();
  for (uint32_t i = t; i < R; i += THREADS) st_l2(&offsets[sb.gA + i], 0u);
  __threadfence();
  __syncthreads();
  for (uint32_t e = t; e < m; e += THREADS) atomicAdd(&offsets[bucket_of(in[sb.kA + e], log2P, sd)], 1u);
  __threadfence();
  __syncthreads();
  uint32_t carry = sb.kA;
  for (uint32_t c0 = 0; c0 < R; c0 += THREADS) {
    const uint32_t i = c0 + t;
    const uint32_t x = i < R ? ld_l2(&offsets[sb.gA + i]) : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_sum<THREADS>(x, wsum, total);
    if (i < R) st_l2(&offsets[sb.gA + i], carry + ex);
    carry += total;
  }
  __threadfence();
  __syncthreads();
  for (uint32_t e = t; e < m; e += THREADS) {
    const K key = in[sb.kA + e];
    const uint32_t p = atomicAdd(&offsets[bucket_of(key, log2P, sd)], 1u);
    out[p] = key;
  }
  __threadfence();
  __syncthreads();
  // Each counter now holds the start of the next bucket: shift by one.
  for (uint32_t c1 = R; c1 > 0;) {
    const uint32_t c0 = c1 > THREADS ? c1 - THREADS : 0u;
    const uint32_t i = c0 + t;
    uint32_t val = 0;
    if (i < c1) val = i == 0 ? sb.kA : ld_l2(&offsets[sb.gA + i - 1]);
    __syncthreads();
    if (i < c1) st_l2(&offsets[sb.gA + i], val);
    __threadfence();
    __syncthreads();
    c1 = c0;
  }
  for (uint32_t i = t; i < R; i += THREADS) {
    const uint32_t e0 = ld_l2(&offsets[sb.gA + i]);
    const uint32_t e1 = i + 1 < R ? ld_l2(&offsets[sb.gA + i + 1]) : sb.kB;
    if (e1 - e0 > kLongT) note_long(long_count, long_list, sb.gA + i, e1 - e0);
  }
}

// The long buckets of the sub-bins k_lds_build flagged (32-bit keys, sub-bins
// of at most kWideR buckets): one workgroup per flagged sub-bin reads the
// bucket starts the build wrote and lists the sub-bin's long buckets with
// one reservation per end of the list (atomics on one address are served one
// at a time: one per wave cost a skewed 2^28 build 2.9 ms).  Thread t takes
// buckets t + k THREADS; the front and back numbers travel packed in one
// word through the workgroup scan (at most kWideR each).
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_note_long(const SegPlan* __restrict__ plan,
                                                       const uint32_t* __restrict__ scan2,
                                                       const uint32_t* __restrict__ offsets,
                                                       const uint32_t* __restrict__ flags,
                                                       uint32_t* __restrict__ long_count,
                                                       uint32_t* __restrict__ long_list) {
  constexpr int CPT = static_cast<int>(kWideR) / THREADS;
  static_assert(CPT * THREADS == static_cast<int>(kWideR) && CPT <= 16 && kWideR < 65536, "one mask word");
  __shared__ uint32_t wtot[THREADS / kWave];
  __shared__ uint32_t base[2];
  __shared__ uint64_t sflagged;
  const uint32_t t = threadIdx.x;
  const uint32_t nsb = plan->total_subbins;
  // This workgroup's sub-bins are blockIdx.x + k gridDim.x; the first wave
  // reads the flags of 64 of them in one load, and the workgroup then visits
  // only the flagged ones (a table without long buckets costs one round trip
  // per workgroup and group of 64).
  for (uint32_t k0 = 0; blockIdx.x + k0 * gridDim.x < nsb; k0 += kWave) {
    if (t < kWave) {
      const uint32_t b = blockIdx.x + (k0 + t) * gridDim.x;
      const uint64_t m = ballot(b < nsb && flags[b] != 0);
      if (t == 0) sflagged = m;
    }
    __syncthreads();
    uint64_t todo = sflagged;
    __syncthreads();  // sflagged is free for the next group
    for (; todo != 0; todo &= todo - 1) {
      const uint32_t kb = k0 + static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(todo)) - 1);
      const uint32_t b = blockIdx.x + kb * gridDim.x;
      const SubBin sb = sub_bin<false>(plan, scan2, b);
      const uint32_t R = sb.gB - sb.gA;
      uint32_t marks = 0;  // bit k: bucket t + k THREADS goes to the front; bit 16 + k: to the back
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        const uint32_t i = t + static_cast<uint32_t>(k) * THREADS;
        if (i < R) {
          const uint32_t len = (i + 1 < R ? offsets[sb.gA + i + 1] : sb.kB) - offsets[sb.gA + i];
          marks |= ((len > kLongT && len <= kWaveLong) ? 1u : 0u) << k;
          marks |= (len > kWaveLong ? 1u : 0u) << (16 + k);
        }
      }
      const uint32_t own =
          static_cast<uint32_t>(__popc(marks & 0xFFFFu)) | (static_cast<uint32_t>(__popc(marks >> 16)) << 16);
      uint32_t total;
      const uint32_t ex = block_exclusive_sum<THREADS>(own, wtot, total);
      if (t == 0) {
        base[0] = (total & 0xFFFFu) != 0 ? atomicAdd(&long_count[0], total & 0xFFFFu) : 0u;
        base[1] = (total >> 16) != 0 ? atomicAdd(&long_count[2], total >> 16) : 0u;
      }
      __syncthreads();
      uint32_t f = base[0] + (ex & 0xFFFFu), bk = base[1] + (ex >> 16);
      const uint32_t cap = long_count[4];
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        const uint32_t g = sb.gA + t + static_cast<uint32_t>(k) * THREADS;
        if ((marks >> k) & 1u) long_list[f++] = g;
        if ((marks >> (16 + k)) & 1u) long_list[cap - 1 - bk++] = g;
      }
      __syncthreads();  // base is free for the next sub-bin
    }
  }
}

// ------------------------------------------------------- heavy sub-bins
// A sub-bin of more than 65535 keys (a few keys of very high multiplicity)
// is built by many workgroups, one chunk of kHeavyChunk keys each, in four
// passes over the queued chunks and sub-bins (persistent grids):
//   count    chunk histogram in LDS, added to the sub-bin's counters;
//   scan     counters -> bucket starts (one workgroup per sub-bin);
//   scatter  chunk histogram again; one global add per bucket reserves the
//            chunk's range; keys written at LDS-counted positions;
//   fix      the counters now hold bucket ends: shift them back into
//            starts and note the long buckets.
// heavy_count[0] = queued chunks, [1] = heavy sub-bins.

template <typename K>
__device__ __forceinline__ void load_sub_bin_desc(PartDesc* sd, const SegPlan* plan, const PartDesc* desc,
                                                  uint32_t seg, uint32_t P, uint32_t threads) {
  const PartDesc* dsrc = plan->desc_by_seg ? desc + seg : desc;
  for (uint32_t i = threadIdx.x; i < P; i += threads) sd[i] = dsrc[i];
}

template <typename K, int THREADS, int REG>
__global__ __launch_bounds__(THREADS) void k_heavy_count(const K* __restrict__ in, const SegPlan* __restrict__ plan,
                                                         const uint32_t* __restrict__ scan2, uint32_t log2P,
                                                         uint32_t P, const PartDesc* __restrict__ desc,
                                                         uint32_t* __restrict__ offsets,
                                                         const uint32_t* __restrict__ heavy_count,
                                                         const uint32_t* __restrict__ heavy_chunks) {
  static_assert(THREADS * REG == kHeavyChunk, "one chunk per pass");
  __shared__ uint32_t hist[kWideR];
  __shared__ PartDesc sd[kMaxP];
  const uint32_t t = threadIdx.x;
  const uint32_t items = heavy_count[0];
  for (uint32_t w = blockIdx.x; w < items; w += gridDim.x) {
    const uint32_t b = heavy_chunks[2 * w], k = heavy_chunks[2 * w + 1];
    const SubBin sb = sub_bin<false>(plan, scan2, b);
    const uint32_t R = sb.gB - sb.gA;
    const uint32_t c0 = sb.kA + k * kHeavyChunk, c1 = min(sb.kB, c0 + kHeavyChunk);
    __syncthreads();  // the previous chunk is done with hist and sd
    load_sub_bin_desc<K>(sd, plan, desc, sb.seg, P, THREADS);
    for (uint32_t i = t; i < R; i += THREADS) hist[i] = 0;
    __syncthreads();
    // Every load in flight at once: a lane past the chunk's end re-reads its
    // last key (c1 > c0) and adds nothing.
    K v[REG];
#pragma unroll
    for (int j = 0; j < REG; ++j) v[j] = in[min(c0 + static_cast<uint32_t>(j) * THREADS + t, c1 - 1)];
#pragma unroll
    for (int j = 0; j < REG; ++j) {
      const uint32_t e = c0 + static_cast<uint32_t>(j) * THREADS + t;
      lds_agg_add<false>(hist, bucket_of(v[j], log2P, sd) - sb.gA, e < c1);
    }
    __syncthreads();
    for (uint32_t i = t; i < R; i += THREADS)
      if (hist[i] != 0) atomicAdd(&offsets[sb.gA + i], hist[i]);
  }
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_heavy_scan(const SegPlan* __restrict__ plan,
                                                        const uint32_t* __restrict__ scan2,
                                                        uint32_t* __restrict__ offsets,
                                                        const uint32_t* __restrict__ heavy_count,
                                                        const uint32_t* __restrict__ heavy_bins) {
  __shared__ uint32_t c[kWideR];
  __shared__ uint32_t wsum[THREADS / kWave];
  const uint32_t t = threadIdx.x;
  const uint32_t nb = heavy_count[1];
  for (uint32_t j = blockIdx.x; j < nb; j += gridDim.x) {
    const SubBin sb = sub_bin<false>(plan, scan2, heavy_bins[j]);
    const uint32_t R = sb.gB - sb.gA;
    __syncthreads();
    for (uint32_t i = t; i < R; i += THREADS) c[i] = offsets[sb.gA + i];
    __syncthreads();
    lds_exclusive_scan32<THREADS>(c, R, wsum);
    for (uint32_t i = t; i < R; i += THREADS) offsets[sb.gA + i] = sb.kA + c[i];
  }
}

template <typename K, int THREADS, int REG>
__global__ __launch_bounds__(THREADS) void k_heavy_scatter(const K* __restrict__ in, const SegPlan* __restrict__ plan,
                                                           const uint32_t* __restrict__ scan2, uint32_t log2P,
                                                           uint32_t P, const PartDesc* __restrict__ desc,
                                                           uint32_t* __restrict__ offsets, K* __restrict__ out,
                                                           const uint32_t* __restrict__ heavy_count,
                                                           const uint32_t* __restrict__ heavy_chunks) {
  static_assert(THREADS * REG == kHeavyChunk, "one chunk per pass");
  __shared__ uint32_t hist[kWideR];
  __shared__ PartDesc sd[kMaxP];
  const uint32_t t = threadIdx.x;
  const uint32_t items = heavy_count[0];
  for (uint32_t w = blockIdx.x; w < items; w += gridDim.x) {
    const uint32_t b = heavy_chunks[2 * w], k = heavy_chunks[2 * w + 1];
    const SubBin sb = sub_bin<false>(plan, scan2, b);
    const uint32_t R = sb.gB - sb.gA;
    const uint32_t c0 = sb.kA + k * kHeavyChunk, c1 = min(sb.kB, c0 + kHeavyChunk);
    __syncthreads();
    load_sub_bin_desc<K>(sd, plan, desc, sb.seg, P, THREADS);
    for (uint32_t i = t; i < R; i += THREADS) hist[i] = 0;
    __syncthreads();
    K v[REG];
    uint32_t lb[REG];
#pragma unroll
    for (int j = 0; j < REG; ++j) v[j] = in[min(c0 + static_cast<uint32_t>(j) * THREADS + t, c1 - 1)];
#pragma unroll
    for (int j = 0; j < REG; ++j) {
      const uint32_t e = c0 + static_cast<uint32_t>(j) * THREADS + t;
      lb[j] = bucket_of(v[j], log2P, sd) - sb.gA;
      lds_agg_add<false>(hist, lb[j], e < c1);
    }
    __syncthreads();
    // Reserve this chunk's range in every bucket it touches.
    for (uint32_t i = t; i < R; i += THREADS)
      if (hist[i] != 0) hist[i] = atomicAdd(&offsets[sb.gA + i], hist[i]);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < REG; ++j) {
      const uint32_t e = c0 + static_cast<uint32_t>(j) * THREADS + t;
      const uint32_t p = lds_agg_add<true>(hist, lb[j], e < c1);
      if (e < c1) out[p] = v[j];
    }
  }
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_heavy_fix(const SegPlan* __restrict__ plan,
                                                       const uint32_t* __restrict__ scan2,
                                                       uint32_t* __restrict__ offsets,
                                                       const uint32_t* __restrict__ heavy_count,
                                                       const uint32_t* __restrict__ heavy_bins,
                                                       uint32_t* __restrict__ long_count,
                                                       uint32_t* __restrict__ long_list) {
  __shared__ uint32_t c[kWideR];
  const uint32_t t = threadIdx.x;
  const uint32_t nb = heavy_count[1];
  for (uint32_t j = blockIdx.x; j < nb; j += gridDim.x) {
    const SubBin sb = sub_bin<false>(plan, scan2, heavy_bins[j]);
    const uint32_t R = sb.gB - sb.gA;
    __syncthreads();
    for (uint32_t i = t; i < R; i += THREADS) c[i] = offsets[sb.gA + i];  // bucket ends
    __syncthreads();
    for (uint32_t i = t; i < R; i += THREADS) {
      const uint32_t start = i == 0 ? sb.kA : c[i - 1];
      offsets[sb.gA + i] = start;
      if (c[i] - start > kLongT) note_long(long_count, long_list, sb.gA + i, c[i] - start);
    }
  }
}

// ------------------------------------------------------------- LDS probe
// Queued chunks of a probe sub-bin hold kProbeQueueLoads register loads of
// queries each (one window set-up per chunk).
constexpr uint32_t kProbeQueueLoads = 4;

// The probe's queue: for every sub-bin with more than ch queries, its
// queries after the first ch in chunks of kProbeQueueLoads * ch, as
// (sub-bin, chunk) pairs after the count queue[0] (zeroed before).  No more
// items than chunks of ch would make: the queue holds q / ch + 1 of them.
__global__ __launch_bounds__(256) void k_probe_queue(const SegPlan* __restrict__ qplan,
                                                     const uint32_t* __restrict__ qscan2, uint32_t ch,
                                                     uint32_t* __restrict__ queue) {
  const uint32_t b = blockIdx.x * 256u + threadIdx.x;
  if (b >= qplan->total_subbins) return;
  const SubBin sb = sub_bin<false>(qplan, qscan2, b);
  const uint32_t m = sb.kB - sb.kA, chq = kProbeQueueLoads * ch;
  if (m <= ch) return;
  const uint32_t extra = (m - ch + chq - 1) / chq;
  const uint32_t at = atomicAdd(&queue[0], extra);
  for (uint32_t k = 0; k < extra; ++k) {
    queue[1 + 2 * (at + k)] = b;
    queue[2 + 2 * (at + k)] = k + 1;
  }
}
// dst[0 .. len) = src[0 .. len), U loads in flight per thread before their
// LDS stores (one wait per batch instead of one per element).
template <int THREADS, int U, typename T>
__device__ __forceinline__ void copy_to_lds(T* __restrict__ dst, const T* __restrict__ src, uint32_t len) {
  const uint32_t t = threadIdx.x;
  for (uint32_t b = 0; b < len; b += THREADS * U) {
    T x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = b + static_cast<uint32_t>(u) * THREADS + t;
      if (i < len) x[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = b + static_cast<uint32_t>(u) * THREADS + t;
      if (i < len) dst[i] = x[u];
    }
  }
}

constexpr uint32_t kProbeKeyBytes = 40 * 1024;
// Offsets and keys of a probe window share one LDS block: the offsets take
// Wb + 1 words, rounded up to 16 bytes, and the keys the rest.  A window of
// fewer than 2^kMaxLog2W buckets (64-bit keys, or several keys per bucket)
// so holds more keys than kProbeKeyBytes, which is what a window whose heavy
// bucket overflows the expected count needs.
constexpr uint32_t kProbeOffWords = (1u << kMaxLog2W) + 4;
constexpr uint32_t kProbeLdsWords = kProbeOffWords + kProbeKeyBytes / 4 + 8;
static_assert(kProbeLdsWords < (1u << 16), "compacted key positions of a window fit 16 bits");

template <typename K, int THREADS, int REG, int MINW>
__global__ __launch_bounds__(THREADS, MINW) void k_lds_probe(const K* __restrict__ q2,
                                                             const SegPlan* __restrict__ qplan,
                                                             const uint32_t* __restrict__ qscan2, uint32_t log2P,
                                                             uint32_t P, const PartDesc* __restrict__ desc,
                                                             const uint32_t* __restrict__ offsets,
                                                             const K* __restrict__ tkeys,
                                                             const uint32_t* __restrict__ unsorted, uint32_t log2W,
                                                             const uint32_t* __restrict__ queue,
                                                             uint32_t max_queued, void* __restrict__ c2v) {
  constexpr uint32_t KCAP = kProbeKeyBytes / sizeof(K);  // keys in LDS at the largest window
  __shared__ __align__(16) uint32_t sbuf[kProbeLdsWords];
  static_assert((kProbeLdsWords - kProbeOffWords) * 4 / sizeof(K) - 4 >= KCAP, "the largest window keeps KCAP keys");
  __shared__ PartDesc sd[kMaxP];
  __shared__ uint32_t nwl;
  const uint32_t t = threadIdx.x;
  // Workgroup w < max_queued takes queued item w (k_probe_queue listed the
  // rest of every sub-bin with more than CH queries, in chunks of CHQ);
  // workgroup max_queued + b takes the first CH queries of sub-bin b.  The
  // long queued chunks (a heavy key's sub-bin) start first, and the short
  // sub-bins fill in around them in the same launch.
  constexpr uint32_t CH = THREADS * REG;
  constexpr uint32_t CHQ = kProbeQueueLoads * CH;
  uint32_t b, chunk;
  if (blockIdx.x < max_queued) {
    const uint32_t w = blockIdx.x;
    if (w >= ld_uniform(queue, 0)) return;  // whole workgroup
    b = ld_uniform(queue, 1 + 2 * w);
    chunk = ld_uniform(queue, 2 + 2 * w);
  } else {
    b = blockIdx.x - max_queued;
    if (b >= qplan->total_subbins) return;  // whole workgroup
    chunk = 0;
  }
  const SubBin sb = sub_bin<true>(qplan, qscan2, b);
  const uint32_t qa = sb.kA + min(chunk == 0 ? 0u : CH + (chunk - 1) * CHQ, sb.kB - sb.kA);
  const uint32_t R = sb.gB - sb.gA, m = min(chunk == 0 ? CH : CHQ, sb.kB - qa);
  const uint32_t Wb = 1u << log2W;
  const uint32_t nuns = unsorted[0];
  // Counts leave as bytes when the table has no long bucket (every count is
  // then at most kLongT), else as u32.
  const bool narrow = unsorted[kHasLongWord] == 0;
  uint8_t* const c2b = static_cast<uint8_t*>(c2v);
  uint32_t* const c2 = static_cast<uint32_t*>(c2v);
  // Keys at the block's start (a fixed address, as the counting loops read
  // them), offsets at its end.
  const uint32_t off_words = (Wb + 4) & ~3u;  // log2W <= kMaxLog2W: at most kProbeOffWords
  uint32_t* const soff = sbuf + (kProbeLdsWords - off_words);
  K* const skeys = reinterpret_cast<K*>(sbuf);
  // 4 spare entries: count_short reads 4 keys of any bucket.
  const uint32_t kcap = (kProbeLdsWords - off_words) * 4 / static_cast<uint32_t>(sizeof(K)) - 4;
  {
    const PartDesc* dsrc = qplan->desc_by_seg ? desc + sb.seg : desc;
    for (uint32_t i = t; i < P; i += THREADS) sd[i] = dsrc[i];
  }
  __syncthreads();

  if (R <= Wb) {
    // The whole sub-bin is one window.  Its offsets, its keys and the first
    // queries are all requested before any of them is waited on (one memory
    // round trip per workgroup instead of one per array); the key range comes
    // from two uniform loads.  Lanes past an array's end re-read its last
    // element and store nothing.
    if (m == 0) return;  // whole workgroup
    constexpr int kUO = ((1u << kMaxLog2W) + THREADS) / THREADS;  // R + 1 <= 2^kMaxLog2W + 1 offsets
    constexpr int kUK = (KCAP + THREADS - 1) / THREADS;
    constexpr int kUQ = REG / 2;  // queries requested per thread and round
    uint32_t xo[kUO];
    K xk[kUK], qv[kUQ];
#pragma unroll
    for (int u = 0; u < kUO; ++u) xo[u] = offsets[sb.gA + min(static_cast<uint32_t>(u) * THREADS + t, R)];
#pragma unroll
    for (int u = 0; u < kUQ; ++u) qv[u] = q2[qa + min(static_cast<uint32_t>(u) * THREADS + t, m - 1)];
    // The key loads wait for the key range; the loads above are in flight
    // meanwhile.
    const uint32_t ka = offsets[sb.gA], nk = offsets[sb.gB] - ka;
    const bool in_lds = nk <= kcap;
    const bool load_keys = in_lds && nk > 0;
    if (load_keys) {
#pragma unroll
      for (int u = 0; u < kUK; ++u) xk[u] = tkeys[ka + min(static_cast<uint32_t>(u) * THREADS + t, nk - 1)];
    }
#pragma unroll
    for (int u = 0; u < kUO; ++u) {
      const uint32_t i = static_cast<uint32_t>(u) * THREADS + t;
      if (i <= R) soff[i] = xo[u];
    }
    if (load_keys) {
#pragma unroll
      for (int u = 0; u < kUK; ++u) {
        const uint32_t i = static_cast<uint32_t>(u) * THREADS + t;
        if (i < nk) skeys[i] = xk[u];
      }
      // Keys past the registers' share (a window smaller than 2^kMaxLog2W).
      for (uint32_t i = kUK * THREADS + t; i < nk; i += THREADS) skeys[i] = tkeys[ka + i];
    }
    __syncthreads();
    // Keys that do not fit LDS mean long buckets (more than kLongT keys).  Up
    // to kWinLong of them are listed in bucket order with their key ranges,
    // and one wave per sorted one finds each run's end by 64-way search and
    // keeps the runs (at most kSetMax) in LDS.  When every long bucket is
    // listed and the short buckets' keys fit beside those tables, they are
    // staged too, compacted: the offsets are rewritten to compacted
    // positions, with kLongMark on a long bucket's own offset.  Only queries
    // into a long bucket without runs then read global memory.
    constexpr uint32_t kWinLong = 32;
    uint32_t* lbkt = reinterpret_cast<uint32_t*>(skeys);  // window bucket of each long bucket, ascending
    uint32_t* lnr = lbkt + kWinLong;                      // its runs, or kOver
    uint32_t* llo = lnr + kWinLong;                       // its key range in the table
    uint32_t* lhi = llo + kWinLong;
    uint32_t* rcnt = lhi + kWinLong;  // [kWinLong][kSetMax] run lengths
    K* rkey = reinterpret_cast<K*>(rcnt + kWinLong * kSetMax);
    constexpr uint32_t kTableBytes = (4 * kWinLong + kWinLong * kSetMax) * 4 + kWinLong * kSetMax * sizeof(K);
    static_assert(kTableBytes % sizeof(K) == 0 && kTableBytes <= KCAP * sizeof(K), "run tables fit the key area");
    K* const sshort = skeys + kTableBytes / sizeof(K);  // staged short-bucket keys
    constexpr uint32_t kLongMark = 0x80000000u;
    uint32_t nl = 0;
    bool staged = false;
    if (!in_lds) {
      if (t == 0) nwl = 0;
      __syncthreads();
      for (uint32_t b = t; b < R; b += THREADS) {
        if (soff[b + 1] - soff[b] > kLongT) {
          const uint32_t s = atomicAdd(&nwl, 1u);
          if (s < kWinLong) lbkt[s] = b;
        }
      }
      __syncthreads();
      const uint32_t nall = wave_uniform(nwl);
      nl = min(nall, kWinLong);
      // Bucket order: thread s ranks the s-th listed bucket among the others.
      uint32_t mine = 0, rank = 0;
      if (t < nl) {
        mine = lbkt[t];
        for (uint32_t j = 0; j < nl; ++j) rank += lbkt[j] < mine ? 1u : 0u;
      }
      __syncthreads();
      if (t < nl) {
        lbkt[rank] = mine;
        llo[rank] = soff[mine];
        lhi[rank] = soff[mine + 1];
      }
      __syncthreads();
      const uint32_t w = t / kWave, l = lane_id();
      for (uint32_t s = w; s < nl; s += THREADS / kWave) {
        const uint32_t b = wave_uniform(lbkt[s]), hi = wave_uniform(lhi[s]);
        uint32_t p = wave_uniform(llo[s]), nr = 0;
        if (long_bucket_sorted(unsorted, nuns, sb.gA + b, kMaxUnsorted)) {
          while (p < hi && nr < kSetMax) {
            const K v = tkeys[p];
            // tkeys[lo2] == v; the run ends in (lo2, h2].
            uint32_t lo2 = p, h2 = hi;
            while (h2 - lo2 > 1) {
              const uint32_t step = (h2 - lo2 + kWave - 1) / kWave;
              const uint32_t pos = lo2 + (l + 1) * step;
              const uint32_t c = popc64(ballot(pos < h2 && tkeys[pos] == v));
              const uint32_t nlo = lo2 + c * step;
              h2 = min(h2, nlo + step);
              lo2 = nlo;
            }
            if (l == 0) {
              rkey[s * kSetMax + nr] = v;
              rcnt[s * kSetMax + nr] = h2 - p;
            }
            ++nr;
            p = h2;
          }
        }
        if (l == 0) lnr[s] = p < hi ? kOver : nr;
      }
      uint32_t nlong = 0;  // keys of the listed long buckets
      for (uint32_t s = 0; s < nl; ++s) nlong += lhi[s] - llo[s];
      const uint32_t cap_short = kcap - kTableBytes / static_cast<uint32_t>(sizeof(K));  // 4 spare kept
      staged = wave_uniform(nall <= kWinLong && nk - nlong <= cap_short ? 1u : 0u) != 0;
      if (staged) {
        // Offsets in compacted positions (below 2^16): less the window's
        // first key and the keys of the long buckets before the bucket.  A
        // long bucket's own offset also carries kLongMark and its list slot
        // in bits 16.., so a query finds its runs without a search.
        for (uint32_t b = t; b <= R; b += THREADS) {
          uint32_t before = 0, mark = 0;
          for (uint32_t s = 0; s < nl; ++s) {
            const uint32_t g = lbkt[s];
            before += g < b ? lhi[s] - llo[s] : 0u;
            mark |= g == b ? (kLongMark | (s << 16)) : 0u;
          }
          soff[b] = (soff[b] - ka - before) | mark;
        }
        // The short buckets' keys: the stretches around the long buckets.
        uint32_t from = ka, to = 0;
        for (uint32_t s = 0; s <= nl; ++s) {
          const uint32_t end = s < nl ? wave_uniform(llo[s]) : ka + nk;
          for (uint32_t i = t; i < end - from; i += THREADS) sshort[to + i] = tkeys[from + i];
          to += end - from;
          if (s < nl) from = wave_uniform(lhi[s]);
        }
      }
      __syncthreads();
    }
    // Count of query v.  Mode 0: the window's keys are in LDS; a short bucket
    // (at most kLongT keys, unsorted) is read by count_short, a long one by
    // binary search when sorted.  Mode 1: short buckets staged, long ones
    // listed.  Mode 2: short buckets in global memory.  The loop below is
    // compiled once per mode, so the common case carries none of the others'
    // code.
    auto count_one = [&](K v, auto mode) -> uint32_t {
      constexpr int MODE = decltype(mode)::value;
      const uint32_t lb = bucket_of(v, log2P, sd) - sb.gA;
      const uint32_t lo = soff[lb], hi = soff[lb + 1];
      if (MODE == 0) {
        if (hi - lo <= kLongT) return count_short(skeys, lo - ka, hi - ka, v);
        return count_equal(skeys, lo - ka, hi - ka, v, long_bucket_sorted(unsorted, nuns, sb.gA + lb, kMaxUnsorted));
      }
      if (MODE == 1) {
        if (!(lo & kLongMark)) return count_short(sshort, lo, hi & 0xFFFFu, v);
        // A long bucket: its runs, else its keys in global memory.
        const uint32_t s = (lo >> 16) & 0x7FFFu;
        const uint32_t nr = lnr[s];
        if (nr != kOver) {
          uint32_t c = 0;
          for (uint32_t r = 0; r < nr; ++r)
            if (rkey[s * kSetMax + r] == v) c = rcnt[s * kSetMax + r];
          return c;
        }
        return count_equal(tkeys, llo[s], lhi[s], v, long_bucket_sorted(unsorted, nuns, sb.gA + lb, kMaxUnsorted));
      }
      if (MODE == 2 && hi - lo <= kLongT) return count_equal(tkeys, lo, hi, v, false);
      // A long bucket: its runs, else a scan of its keys in global memory.
      for (uint32_t s = 0; s < nl; ++s) {
        if (lbkt[s] != lb) continue;
        const uint32_t nr = lnr[s];
        if (nr != kOver) {
          uint32_t c = 0;
          for (uint32_t r = 0; r < nr; ++r)
            if (rkey[s * kSetMax + r] == v) c = rcnt[s * kSetMax + r];
          return c;
        }
        return count_equal(tkeys, llo[s], lhi[s], v, long_bucket_sorted(unsorted, nuns, sb.gA + lb, kMaxUnsorted));
      }
      return count_equal(tkeys, lo, hi, v, long_bucket_sorted(unsorted, nuns, sb.gA + lb, kMaxUnsorted));
    };
    // A thread remembers its last query and count: in a sub-bin that holds
    // a heavy key, most of a thread's queries repeat it.
    auto run = [&](auto mode) {
      K last_q = K(0);
      uint32_t last_c = 0;
      bool have = false;
      for (uint32_t c0 = 0;;) {
#pragma unroll
        for (int u = 0; u < kUQ; ++u) {
          const uint32_t e = c0 + static_cast<uint32_t>(u) * THREADS + t;
          if (e < m) {
            if (!have || qv[u] != last_q) {
              last_c = count_one(qv[u], mode);
              last_q = qv[u];
              have = true;
            }
            if (narrow)
              c2b[qa + e] = static_cast<uint8_t>(last_c);
            else
              c2[qa + e] = last_c;
          }
        }
        c0 += THREADS * kUQ;
        if (c0 >= m) break;
#pragma unroll
        for (int u = 0; u < kUQ; ++u) qv[u] = q2[qa + min(c0 + static_cast<uint32_t>(u) * THREADS + t, m - 1)];
      }
    };
    if (in_lds)
      run(std::integral_constant<int, 0>());
    else if (staged)
      run(std::integral_constant<int, 1>());
    else
      run(std::integral_constant<int, 2>());
    return;
  }

  for (uint32_t c0 = 0; c0 < m; c0 += THREADS * REG) {  // one pass unless the sub-bin is oversized
    K qv[REG];
    // Two 16-bit counts per word, saturated at 0xFFFF (such a query is
    // counted again from global memory when the counts are written).
    uint32_t cnt[(REG + 1) / 2];
#pragma unroll
    for (int j = 0; j < REG; ++j) {
      const uint32_t e = c0 + static_cast<uint32_t>(j) * THREADS + t;
      if (e < m) qv[j] = q2[qa + e];
    }
#pragma unroll
    for (int j = 0; j < (REG + 1) / 2; ++j) cnt[j] = 0;
    // Each query's bucket lies in exactly one window: its count is taken
    // when that window is in LDS and written once, after the last window, so
    // every output line leaves whole.
    for (uint32_t w0 = 0; w0 < R; w0 += Wb) {
      const uint32_t wl = min(Wb, R - w0);
      copy_to_lds<THREADS, 8>(soff, offsets + sb.gA + w0, wl + 1);
      __syncthreads();
      const uint32_t ka = soff[0], nk = soff[wl] - ka;
      const bool in_lds = nk <= kcap;
      if (in_lds) copy_to_lds<THREADS, 8>(skeys, tkeys + ka, nk);
      __syncthreads();
      // Output addresses are rebuilt in every window from one register (the
      // empty asm keeps REG 64-bit addresses from being hoisted and spilled).
      uint32_t ebase = c0 + t;
      asm volatile("" : "+v"(ebase));
#pragma unroll
      for (int j = 0; j < REG; ++j) {
        const uint32_t e = ebase + static_cast<uint32_t>(j) * THREADS;
        if (e < m) {
          // Recompute the bucket in every window rather than keep REG of
          // them live: the empty asm stops the compiler from hoisting it.
          asm volatile("" : "+v"(qv[j]));
          const uint32_t lb = bucket_of(qv[j], log2P, sd) - sb.gA;
          if (lb >= w0 && lb < w0 + wl) {
            const uint32_t lo = soff[lb - w0], hi = soff[lb - w0 + 1];
            const bool srt = hi - lo > kLongT && long_bucket_sorted(unsorted, nuns, sb.gA + lb, kMaxUnsorted);
            const uint32_t c = in_lds ? count_equal(skeys, lo - ka, hi - ka, qv[j], srt)
                                      : count_equal(tkeys, lo, hi, qv[j], srt);
            cnt[j >> 1] |= min(c, 0xFFFFu) << ((j & 1) << 4);
          }
        }
      }
      __syncthreads();
    }
    uint32_t fbase = c0 + t;  // (not hoisted above the windows: see ebase)
    asm volatile("" : "+v"(fbase));
#pragma unroll
    for (int j = 0; j < REG; ++j) {
      const uint32_t e = fbase + static_cast<uint32_t>(j) * THREADS;
      if (e < m) {
        uint32_t c = (cnt[j >> 1] >> ((j & 1) << 4)) & 0xFFFFu;
        if (c == 0xFFFFu) {  // a bucket of 65535 keys or more
          const uint32_t g = bucket_of(qv[j], log2P, sd);
          const uint32_t lo = offsets[g], hi = offsets[g + 1];
          c = count_equal(tkeys, lo, hi, qv[j], long_bucket_sorted(unsorted, nuns, g, kMaxUnsorted));
        }
        if (narrow)
          c2b[qa + e] = static_cast<uint8_t>(c);
        else
          c2[qa + e] = c;
      }
    }
  }
}

// --------------------------------------------------------- long buckets
// Buckets with more than kLongT keys are sorted in place, so that a probe
// counts them with two binary searches (the order inside a bucket is free).
// Buckets of at most kWaveLong keys are taken by single waves first
// (k_long_small: runs, or a sort in registers up to wave_sort_max keys);
// the rest, and those a wave could neither rewrite nor sort, take one
// workgroup each, claimed from a work counter (k_long_sort):
//   0. a bucket of at most sort_cap<K>() keys (64 KiB) that no key
//      dominates (key_dominates) is listed for k_long_wgsort at once;
//   1. otherwise the distinct keys of the bucket and their multiplicities,
//      found by leader election in each wave (one round per distinct key in
//      the wave's 64 keys) and merged into a set of at most kSetMax;
//   2. the bucket rewritten as runs of those keys in ascending order (not
//      needed for a single distinct key);
//   3. a bucket with more distinct keys is listed for k_long_wgsort (a
//      bitonic sort in the workgroup's registers) when it has at most
//      sort_cap<K>() keys, and otherwise listed as unsorted.
// A bucket of more than kBigChunk keys is queued instead, in chunks: every
// chunk finds its own distinct keys (k_big_scan), one workgroup per bucket
// merges them and lays out the runs (k_big_fix), and every chunk rewrites
// its range (k_big_write).
template <typename K>
constexpr uint32_t sort_cap() { return 65536u / sizeof(K); }

template <typename K>
__device__ __forceinline__ K readlane_key(K v, uint32_t lane);
template <>
__device__ __forceinline__ uint32_t readlane_key<uint32_t>(uint32_t v, uint32_t lane) {
  return __builtin_amdgcn_readlane(v, lane);
}
template <>
__device__ __forceinline__ uint64_t readlane_key<uint64_t>(uint64_t v, uint32_t lane) {
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(v), lane);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(v >> 32), lane);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// The value of lane (this lane ^ j) (j < 64), through ds_bpermute.
template <typename K>
__device__ __forceinline__ K lane_xor(K v, uint32_t j);
template <>
__device__ __forceinline__ uint32_t lane_xor<uint32_t>(uint32_t v, uint32_t j) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_ds_bpermute(static_cast<int>((lane_id() ^ j) << 2), static_cast<int>(v)));
}
template <>
__device__ __forceinline__ uint64_t lane_xor<uint64_t>(uint64_t v, uint32_t j) {
  const int a = static_cast<int>((lane_id() ^ j) << 2);
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(a, static_cast<int>(static_cast<uint32_t>(v))));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(a, static_cast<int>(static_cast<uint32_t>(v >> 32))));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Bitonic sort, ascending, of the 64 * KPL keys a wave holds in registers:
// element e = 64 r + lane sits in v[r].  A compare-exchange at distance
// 2^lj < 64 pairs lanes (one lane exchange per register), one at 64 or more
// pairs registers of the same lane.  Both exponent loops are unrolled, so
// every register index is a constant.
template <typename K, int KPL>
__device__ __forceinline__ void wave_bitonic(K (&v)[KPL]) {
  constexpr int kLog2N = 6 + (KPL >= 2) + (KPL >= 4) + (KPL >= 8) + (KPL >= 16) + (KPL >= 32);
  static_assert((64 * KPL) == (1 << kLog2N), "KPL is a power of two up to 32");
  const uint32_t l = lane_id();
#pragma unroll
  for (int lk = 1; lk <= kLog2N; ++lk) {
#pragma unroll
    for (int lj = lk - 1; lj >= 0; --lj) {
      if (lj >= 6) {
        const int jr = 1 << (lj - 6);
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          if ((r & jr) == 0) {
            // Elements 64 r + l and 64 (r + jr) + l; the direction bit
            // (element & 2^lk, lk > 6) depends on r alone.
            const bool up = ((r << 6) & (1 << lk)) == 0;
            const K a = v[r], b = v[r + jr];
            const bool sw = (a > b) == up;
            v[r] = sw ? b : a;
            v[r + jr] = sw ? a : b;
          }
        }
      } else {
        const uint32_t j = 1u << lj;
        const bool lower = (l & j) == 0;  // this lane holds the smaller element of its pair
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          const K o = lane_xor<K>(v[r], j);
          const uint32_t e = (static_cast<uint32_t>(r) << 6) | l;
          const bool up = (e & (1u << lk)) == 0;
          // Ascending pairs keep the smaller key in the lower element.
          v[r] = (lower == up) ? (o < v[r] ? o : v[r]) : (o > v[r] ? o : v[r]);
        }
      }
    }
  }
}

// Sorts keys[lo, lo + L) (64 (KPL / 2) < L <= 64 KPL) by one wave: the keys
// are padded with the largest key, sorted in registers and the first L
// written back (padding equals the largest key, so the first L hold the
// bucket's own multiset).
template <typename K, int KPL>
__device__ __forceinline__ void wave_sort_range(K* __restrict__ keys, uint32_t lo, uint32_t L) {
  const uint32_t l = lane_id();
  K v[KPL];
#pragma unroll
  for (int r = 0; r < KPL; ++r) {
    const uint32_t e = (static_cast<uint32_t>(r) << 6) | l;
    v[r] = e < L ? keys[lo + e] : ~K(0);
  }
  wave_bitonic<K, KPL>(v);
#pragma unroll
  for (int r = 0; r < KPL; ++r) {
    const uint32_t e = (static_cast<uint32_t>(r) << 6) | l;
    if (e < L) keys[lo + e] = v[r];
  }
}

// Adds (v, c) to the set of wave-owned slots sv/sc (size *sz, at most cap <=
// kSetMax), the whole wave searching in parallel.  Returns false when the
// set is full.
template <typename K>
__device__ __forceinline__ bool set_add(K* sv, uint32_t* sc, uint32_t* sz, K v, uint32_t c, uint32_t cap = kSetMax) {
  const uint32_t l = lane_id();
  const uint32_t n = wave_uniform(*sz);
  const uint64_t hit = ballot(l < n && sv[l] == v);
  if (hit != 0) {
    if (l == static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(hit)) - 1)) sc[l] += c;
  } else {
    if (n >= cap) return false;
    if (l == 0) {
      sv[n] = v;
      sc[n] = c;
      *sz = n + 1;
    }
  }
  __builtin_amdgcn_wave_barrier();
  return true;
}

// The distinct keys of src[i] for the i in [a, b) that this wave visits
// (groups of 64 from `first`, then every `step`), with multiplicities, added
// to the wave's set sv / sc / *sz.  False when the set overflows (or *stop
// turns nonzero: another wave's set overflowed).  The wave keeps the last
// key it met and that key's pending count in registers, and touches the set
// only when the key changes (a run of one heavy key costs a ballot per 64
// keys); it reads kDistinctGroups groups of 64 keys per round, all loads in
// flight before the first is used.  The set holds at most cap keys.  `pre`,
// when given, holds the first round's keys, already loaded as the loop
// would load them.
constexpr int kDistinctGroups = 8;
template <typename K>
__device__ __forceinline__ bool wave_distinct(const K* __restrict__ src, uint32_t first, uint32_t b, uint32_t step, K* sv,
                              uint32_t* sc, uint32_t* sz, const uint32_t* stop, uint32_t cap = kSetMax,
                              const K* pre = nullptr) {
  constexpr int kGroups = kDistinctGroups;
  const uint32_t l = lane_id();
  K last = K(0);
  uint32_t pend = 0;
  bool ok = true;
  for (uint32_t c0 = first; c0 < b && ok; c0 += step) {
    if (stop != nullptr && wave_uniform(*stop)) return false;
    K kv[kGroups];
    // All kGroups loads in flight: a lane past b re-reads src[b - 1] (c0 < b)
    // and is not valid below.
    if (pre != nullptr && c0 == first) {
#pragma unroll
      for (int gi = 0; gi < kGroups; ++gi) kv[gi] = pre[gi];
    } else {
#pragma unroll
      for (int gi = 0; gi < kGroups; ++gi) kv[gi] = src[min(c0 + gi * kWave + l, b - 1)];
    }
#pragma unroll
    for (int gi = 0; gi < kGroups; ++gi) {
      const uint32_t i = c0 + gi * kWave + l;
      const bool valid = i < b;
      const K key = kv[gi];
      uint64_t active = ballot(valid);
      if (pend != 0) {
        const uint64_t same = ballot(valid && key == last);
        pend += popc64(same);
        active &= ~same;
      }
      while (active != 0 && ok) {
        const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(active)) - 1);
        const K v = readlane_key(key, leader);
        const uint64_t match = ballot(valid && key == v) & active;
        active &= ~match;
        if (pend != 0 && !set_add(sv, sc, sz, last, pend, cap)) {
          ok = false;
          break;
        }
        last = v;
        pend = popc64(match);
      }
    }
  }
  if (ok && pend != 0 && !set_add(sv, sc, sz, last, pend, cap)) ok = false;
  return ok;
}

// The distinct keys of src[a .. b) and their multiplicities, by the whole
// workgroup: each wave builds a set, wave 0 merges them into sval[0] /
// scnt[0] / ssize[0]; *soverflow is set when there are more than kSetMax.
// Every thread calls it; it starts and ends with a barrier.
template <typename K, int THREADS>
__device__ __forceinline__ void wg_distinct(const K* __restrict__ src, uint32_t a, uint32_t b, K (*sval)[kSetMax],
                            uint32_t (*scnt)[kSetMax], uint32_t* ssize, uint32_t* soverflow) {
  constexpr int W = THREADS / kWave;
  constexpr uint32_t kGroup = kWave * 8;
  const uint32_t t = threadIdx.x, w = t / kWave, l = lane_id();
  if (l == 0) ssize[w] = 0;
  if (t == 0) *soverflow = 0;
  __syncthreads();
  const bool ok = wave_distinct<K>(src, a + w * kGroup, b, THREADS * 8, sval[w], scnt[w], &ssize[w], soverflow);
  if (!ok && l == 0) *soverflow = 1;
  __syncthreads();
  if (w == 0 && !wave_uniform(*soverflow)) {
    for (int x = 1; x < W; ++x) {
      const uint32_t nx = wave_uniform(ssize[x]);
      bool full = false;
      for (uint32_t e = 0; e < nx; ++e) {
        if (!set_add(sval[0], scnt[0], &ssize[0], sval[x][e], scnt[x][e])) {
          if (l == 0) *soverflow = 1;
          full = true;
          break;
        }
      }
      if (full) break;
    }
  }
  __syncthreads();
}

// Ranks the nd distinct keys of sval[0] / scnt[0] into ascending order in
// sval[1] / scnt[1] and their run starts into run0[0 .. nd].  Every thread
// calls it (nd <= kSetMax <= THREADS).
template <typename K>
__device__ __forceinline__ void rank_runs(uint32_t nd, K (*sval)[kSetMax], uint32_t (*scnt)[kSetMax], uint32_t* run0) {
  const uint32_t t = threadIdx.x;
  K myv = 0;
  uint32_t myc = 0, rank = 0;
  if (t < nd) {
    myv = sval[0][t];
    myc = scnt[0][t];
    for (uint32_t j = 0; j < nd; ++j) rank += sval[0][j] < myv ? 1u : 0u;
  }
  __syncthreads();
  if (t < nd) {
    sval[1][rank] = myv;
    scnt[1][rank] = myc;
  }
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    for (uint32_t r = 0; r < nd; ++r) {
      run0[r] = run;
      run += scnt[1][r];
    }
    run0[nd] = run;
  }
  __syncthreads();
}

// Workspace of the chunked long buckets (big_words words).
template <typename K>
struct BigWork {
  uint32_t* ctr;        // [0] big buckets, [1] chunks
  uint32_t* big_g;      // bucket id of big bucket b
  uint32_t* big_first;  // its first chunk
  uint32_t* chunk_b;    // big bucket of chunk c
  uint32_t* chunk_k;    // chunk number inside its bucket
  uint32_t* chunk_n;    // distinct keys of chunk c, or kOver
  uint32_t* chunk_cnt;  // [c][kSetMax]
  K* chunk_key;         // [c][kSetMax]
  uint32_t* run_n;      // distinct keys of big bucket b, or kOver
  uint32_t* run0;       // [b][kSetMax + 1] run starts
  K* run_key;           // [b][kSetMax]
};

template <typename K>
BigWork<K> big_work(uint32_t* base, uint64_t n) {
  const uint64_t nb = big_buckets_max(n), nc = 2 * nb;
  auto align8 = [base](uint32_t* p) { return base + (((p - base) + 1) & ~static_cast<ptrdiff_t>(1)); };
  BigWork<K> w;
  uint32_t* p = base;
  w.ctr = p;
  p += 4;
  w.big_g = p;
  p += nb;
  w.big_first = p;
  p += nb;
  w.chunk_b = p;
  p += nc;
  w.chunk_k = p;
  p += nc;
  w.chunk_n = p;
  p += nc;
  w.chunk_cnt = p;
  p += nc * kSetMax;
  p = align8(p);
  w.chunk_key = reinterpret_cast<K*>(p);
  p += nc * kSetMax * (sizeof(K) / 4);
  w.run_n = p;
  p += nb;
  w.run0 = p;
  p += nb * (kSetMax + 1);
  p = align8(p);
  w.run_key = reinterpret_cast<K*>(p);
  return w;
}

// Bitonic sort, ascending, of the THREADS * KPL keys a workgroup holds in
// registers: element e = KPL t + r sits in v[r] of thread t (a thread holds
// KPL consecutive elements).  A compare-exchange at distance j pairs
// registers of one thread (j < KPL), lanes of one wave (j < 64 KPL: one lane
// exchange per register), or threads of different waves (through `lds`, one
// element per slot: every element written, a barrier, the partner read).
// Both exponent loops are unrolled.  Every thread of the workgroup calls it.
template <typename K, int THREADS, int KPL>
__device__ __forceinline__ void wg_bitonic(K (&v)[KPL], K* lds) {
  constexpr int kLog2KPL = (KPL >= 2) + (KPL >= 4) + (KPL >= 8) + (KPL >= 16);
  constexpr int kLog2T = 6 + (THREADS >= 128) + (THREADS >= 256) + (THREADS >= 512) + (THREADS >= 1024);
  constexpr int kLog2N = kLog2KPL + kLog2T;
  static_assert((1 << kLog2KPL) == KPL && (1 << kLog2T) == THREADS, "powers of two");
  const uint32_t l = lane_id();
  const uint32_t base = threadIdx.x * KPL;
#pragma unroll
  for (int lk = 1; lk <= kLog2N; ++lk) {
#pragma unroll
    for (int lj = lk - 1; lj >= 0; --lj) {
      const uint32_t j = 1u << lj;
      if (lj < kLog2KPL) {
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          if ((r & static_cast<int>(j)) == 0) {
            const bool up = ((base + r) & (1u << lk)) == 0;
            const K a = v[r], b = v[r + j];
            const bool sw = (a > b) == up;
            v[r] = sw ? b : a;
            v[r + j] = sw ? a : b;
          }
        }
      } else if (lj < kLog2KPL + 6) {
        const uint32_t jl = j >> kLog2KPL;  // distance in lanes
        const bool lower = (l & jl) == 0;   // this lane holds the smaller elements of its pairs
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          const K o = lane_xor<K>(v[r], jl);
          const bool up = ((base + r) & (1u << lk)) == 0;
          v[r] = (lower == up) ? (o < v[r] ? o : v[r]) : (o > v[r] ? o : v[r]);
        }
      } else {
        __syncthreads();  // the previous exchange's reads are done
#pragma unroll
        for (int r = 0; r < KPL; ++r) lds[base + r] = v[r];
        __syncthreads();
        const bool lower = (base & j) == 0;  // j >= 64 KPL: the same for all r
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          const K o = lds[(base + r) ^ j];
          const bool up = ((base + r) & (1u << lk)) == 0;
          v[r] = (lower == up) ? (o < v[r] ? o : v[r]) : (o > v[r] ? o : v[r]);
        }
      }
    }
  }
}

// Sorts keys[lo, lo + L) (L <= THREADS KPL) by the workgroup: the keys are
// padded with the largest key, sorted in registers and the first L written
// back.  `lds` holds THREADS KPL keys.  Every thread calls it.
template <typename K, int THREADS, int KPL>
__device__ __forceinline__ void wg_sort_range(K* __restrict__ keys, uint32_t lo, uint32_t L, K* lds) {
  const uint32_t base = threadIdx.x * KPL;
  K v[KPL];
#pragma unroll
  for (int r = 0; r < KPL; ++r) v[r] = base + r < L ? keys[lo + base + r] : ~K(0);
  wg_bitonic<K, THREADS, KPL>(v, lds);
#pragma unroll
  for (int r = 0; r < KPL; ++r)
    if (base + r < L) keys[lo + base + r] = v[r];
}

// Whether one key dominates a bucket: at least half of the 64 keys in kv
// (its first 64, lane l holding key l) equal the key of lane 0, 21 or 42 (a
// heavy key and a few others; three candidates, so that a rare key in lane 0
// does not hide it).  Uniform over the wave.
template <typename K>
__device__ __forceinline__ bool key_dominates(K kv) {
  const uint32_t m0 = popc64(ballot(kv == readlane_key(kv, 0)));
  const uint32_t m1 = popc64(ballot(kv == readlane_key(kv, 21)));
  const uint32_t m2 = popc64(ballot(kv == readlane_key(kv, 42)));
  return max(m0, max(m1, m2)) >= kWave / 2;
}

// Long buckets of up to this many keys are sorted by one wave in registers
// when no key dominates them (64 KPL keys per lane, KPL <= 32 for 32-bit
// keys and <= 16 for 64-bit ones).
template <typename K>
constexpr uint32_t wave_sort_max() { return sizeof(K) == 4 ? 2048u : 1024u; }
constexpr uint32_t kListDone = 0xFFFFFFFFu;  // a front-list entry the runs instance finished
constexpr int kLongWaveThreads = 256;

// Sorts keys[lo, lo + L) by one wave (kLongT < L <= wave_sort_max<K>()).
template <typename K>
__device__ __forceinline__ void wave_sort_bucket(K* __restrict__ keys, uint32_t lo, uint32_t L) {
  if (L <= 128)
    wave_sort_range<K, 2>(keys, lo, L);
  else if (L <= 256)
    wave_sort_range<K, 4>(keys, lo, L);
  else if (L <= 512)
    wave_sort_range<K, 8>(keys, lo, L);
  else if (L <= 1024)
    wave_sort_range<K, 16>(keys, lo, L);
  else if constexpr (wave_sort_max<K>() >= 2048)
    wave_sort_range<K, 32>(keys, lo, L);
}

// Long buckets of at most kWaveLong keys (the front of the list), one wave
// each, in two launches over the same list.  !SORT (first): buckets in which
// one key dominates (key_dominates), or longer than wave_sort_max<K>(); their
// distinct keys are found by ballots, up to kSetMax, and the bucket is
// rewritten as their runs in ascending order by the whole wave, or, with
// more, moves to the back of the list (the workgroups of k_long_sort).  Its
// entries are then marked done.  SORT: every entry not marked, sorted by the
// wave in registers; a wave reads 64 entries per load and passes the marked
// ones by a ballot.  The sorting instance's registers thus lower neither the
// occupancy of the other nor the cost of passing its entries.
template <typename K, int THREADS, bool SORT>
__global__ __launch_bounds__(THREADS, SORT ? 4 : 1) void k_long_small(const uint32_t* __restrict__ offsets,
                                                                    uint32_t* __restrict__ ctr,
                                                                    uint32_t* __restrict__ list, K* __restrict__ keys,
                                                                    uint32_t* __restrict__ unsorted) {
  constexpr int W = THREADS / kWave;
  __shared__ K sval[W][kSetMax];
  __shared__ uint32_t scnt[W][kSetMax];
  __shared__ uint32_t ssize[W];
  const uint32_t w = threadIdx.x / kWave, l = lane_id();
  const uint32_t total = ctr[0];
  // Whether the table has a long bucket: some bucket was listed, at the
  // front (ctr[0], not changed here) or at the back (ctr[2], which the
  // !SORT instance only raises, and only when ctr[0] is nonzero).
  if (!SORT && blockIdx.x == 0 && threadIdx.x == 0) unsorted[kHasLongWord] = (total | ctr[2]) != 0 ? 1u : 0u;
  const uint32_t waves = gridDim.x * W;
  if (SORT) {
    // Wave i reads entries 64 i .. 64 i + 63, then 64 (i + waves) .., in one
    // load each, and sorts the buckets not marked done one after another.
    for (uint32_t c0 = (blockIdx.x * W + wave_uniform(w)) * kWave; c0 < total; c0 += waves * kWave) {
      const uint32_t gl = c0 + l < total ? list[c0 + l] : kListDone;
      for (uint64_t todo = ballot(gl != kListDone); todo != 0; todo &= todo - 1) {
        const uint32_t g = readlane(gl, static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(todo)) - 1));
        // Uniform over the wave: the sort's lane exchanges need every lane.
        const uint32_t lo = wave_uniform(offsets[g]), L = wave_uniform(offsets[g + 1]) - lo;
        wave_sort_bucket<K>(keys, lo, L);
      }
    }
    return;
  }
  // Wave i takes list entries i, i + (waves in the grid), ...: no claims
  // through a shared counter (the buckets are at most kWaveLong keys, so a
  // fixed deal stays balanced).  The loop is uniform over the wave.
  for (uint32_t idx = blockIdx.x * W + wave_uniform(w); idx < total; idx += waves) {
    const uint32_t g = wave_uniform(list[idx]);
    const uint32_t lo = wave_uniform(offsets[g]), L = wave_uniform(offsets[g + 1]) - lo;
    // The distinct search's first round of keys, loaded once: its first 64
    // keys also decide whether one key dominates.
    K kv0[kDistinctGroups];
#pragma unroll
    for (int gi = 0; gi < kDistinctGroups; ++gi) kv0[gi] = keys[lo + min(gi * kWave + l, L - 1)];
    const bool heavy = key_dominates<K>(kv0[0]);
    if (L <= wave_sort_max<K>() && !heavy) continue;  // the sorting instance's bucket
    if (l == 0) {
      ssize[w] = 0;
      list[idx] = kListDone;  // read only by the sorting instance, after this kernel
    }
    __builtin_amdgcn_wave_barrier();
    // A longer bucket no key dominates goes to the back at once (its many
    // distinct keys would overflow the set; k_long_sort sorts it).
    if (!heavy || !wave_distinct<K>(keys + lo, 0, L, kWave * kDistinctGroups, sval[w], scnt[w], &ssize[w], nullptr,
                                     kSetMax, kv0)) {
      if (l == 0) list[ctr[4] - 1 - atomicAdd(&ctr[2], 1u)] = g;
      continue;
    }
    const uint32_t nd = wave_uniform(ssize[w]);
    if (nd <= 1) continue;  // one run already
    // Lane e < nd holds distinct key e; its run starts after the smaller keys.
    const K v = l < nd ? sval[w][l] : K(0);
    const uint32_t c = l < nd ? scnt[w][l] : 0u;
    uint32_t start = 0;
    for (uint32_t j = 0; j < nd; ++j) start += sval[w][j] < v ? scnt[w][j] : 0u;
    for (uint32_t e = 0; e < nd; ++e) {
      const uint32_t rs = readlane(start, e), rc = readlane(c, e);
      const K key = readlane_key(v, e);
      for (uint32_t i = l; i < rc; i += kWave) keys[lo + rs + i] = key;
    }
  }
}

template <typename K>
__global__ __launch_bounds__(kLongThreads) void k_long_sort(const uint32_t* __restrict__ offsets,
                                                            uint32_t* __restrict__ ctr,
                                                            uint32_t* __restrict__ list, K* __restrict__ keys,
                                                            uint32_t* __restrict__ unsorted, BigWork<K> bw) {
  constexpr int W = kLongThreads / kWave;
  __shared__ K sval[W][kSetMax];
  __shared__ uint32_t scnt[W][kSetMax];
  __shared__ uint32_t ssize[W];
  __shared__ uint32_t run0[kSetMax + 1];
  __shared__ uint32_t soverflow;
  __shared__ uint32_t sidx;
  constexpr uint32_t kClaimMax = 16;
  __shared__ uint32_t sortq[kClaimMax];  // this claim's buckets for the register sort
  __shared__ uint32_t nsortq, sbase;
  const uint32_t t = threadIdx.x;
  const uint32_t total = ctr[2], cap = ctr[4];
  // Buckets are claimed `claim` at a time, and a claim's buckets for the
  // register sort are listed with one atomic: atomics on one address are
  // served one at a time, and a table of long buckets lists tens of
  // thousands here.  A short list (a few large buckets) is dealt one by one.
  const uint32_t claim = min(kClaimMax, max(1u, total / (gridDim.x * 8u)));
  for (;;) {
    if (t == 0) {
      sidx = atomicAdd(&ctr[3], claim);
      nsortq = 0;
    }
    __syncthreads();
    const uint32_t idx0 = wave_uniform(sidx);
    if (idx0 >= total) break;  // uniform: every thread read the same sidx
    const uint32_t idx1 = min(idx0 + claim, total);
    for (uint32_t idx = idx0; idx < idx1; ++idx) {
      const uint32_t g = wave_uniform(list[cap - 1 - idx]);
      const uint32_t lo = wave_uniform(offsets[g]), L = wave_uniform(offsets[g + 1]) - lo;
      if (L > kBigChunk) {
        // Queued in chunks for the workgroups of k_big_scan.
        if (t == 0) {
          const uint32_t b = atomicAdd(&bw.ctr[0], 1u);
          const uint32_t nch = (L + kBigChunk - 1) / kBigChunk;
          const uint32_t at = atomicAdd(&bw.ctr[1], nch);
          bw.big_g[b] = g;
          bw.big_first[b] = at;
          for (uint32_t k = 0; k < nch; ++k) {
            bw.chunk_b[at + k] = b;
            bw.chunk_k[at + k] = k;
          }
        }
        __syncthreads();
        continue;
      }
      if (L <= sort_cap<K>()) {
        // No key dominates (every wave tests the same first 64 keys): on to
        // the register sort at once, without a distinct search.
        if (!key_dominates<K>(keys[lo + min(lane_id(), L - 1)])) {
          if (t == 0) sortq[nsortq++] = g;
          __syncthreads();
          continue;
        }
      }
      wg_distinct<K, kLongThreads>(keys + lo, 0, L, sval, scnt, ssize, &soverflow);
      const bool over = wave_uniform(soverflow) != 0;
      const uint32_t nd0 = wave_uniform(ssize[0]);
      if (!over && nd0 <= 1) {
        // one distinct key: the bucket is already one run
      } else if (!over) {
        // rank the distinct keys, then rewrite the bucket as ascending runs
        const uint32_t nd = nd0;
        rank_runs<K>(nd, sval, scnt, run0);
        // Positions only grow along a thread's loop: walk the run index.
        uint32_t a = 0;
        for (uint32_t i = t; i < L; i += kLongThreads) {
          while (a + 1 < nd && run0[a + 1] <= i) ++a;
          keys[lo + i] = sval[1][a];
        }
      } else if (L <= sort_cap<K>()) {
        // many distinct keys, few enough for a workgroup's registers
        if (t == 0) sortq[nsortq++] = g;
      } else if (t == 0) {
        const uint32_t u = atomicAdd(&unsorted[0], 1u);
        if (u < kMaxUnsorted) unsorted[1 + u] = g;
      }
      __syncthreads();
    }
    // The claim's buckets for k_long_wgsort, in the list's free middle
    // (after the ctr[0] front entries; the back's ctr[2] entries leave room).
    const uint32_t nq = wave_uniform(nsortq);
    if (t == 0 && nq != 0) sbase = atomicAdd(&ctr[5], nq);
    __syncthreads();
    if (t < nq) list[ctr[0] + sbase + t] = sortq[t];
    __syncthreads();  // sidx, sortq and its count are free for the next claim
  }
}

// The buckets k_long_sort listed (no dominant key, or more than kSetMax
// distinct keys; at most sort_cap<K>() keys): one workgroup each, sorted in
// registers (wg_bitonic; the exchanges across waves go through LDS).  A
// kernel of its own, so that its registers do not lower the occupancy of
// k_long_sort.
template <typename K>
__global__ __launch_bounds__(kLongThreads) void k_long_wgsort(const uint32_t* __restrict__ offsets,
                                                              const uint32_t* __restrict__ ctr,
                                                              const uint32_t* __restrict__ list,
                                                              K* __restrict__ keys) {
  __shared__ K sbuf[sort_cap<K>()];
  const uint32_t total = ctr[5], first = ctr[0];
  for (uint32_t idx = blockIdx.x; idx < total; idx += gridDim.x) {
    const uint32_t g = wave_uniform(list[first + idx]);
    const uint32_t lo = wave_uniform(offsets[g]), L = wave_uniform(offsets[g + 1]) - lo;
    if (L <= kLongThreads)
      wg_sort_range<K, kLongThreads, 1>(keys, lo, L, sbuf);
    else if (L <= 2 * kLongThreads)
      wg_sort_range<K, kLongThreads, 2>(keys, lo, L, sbuf);
    else if (L <= 4 * kLongThreads)
      wg_sort_range<K, kLongThreads, 4>(keys, lo, L, sbuf);
    else if (L <= 8 * kLongThreads)
      wg_sort_range<K, kLongThreads, 8>(keys, lo, L, sbuf);
    else if constexpr (sort_cap<K>() >= 16 * kLongThreads)
      wg_sort_range<K, kLongThreads, 16>(keys, lo, L, sbuf);
    __syncthreads();  // sbuf is free for the next bucket
  }
}

// Every queued chunk of a big bucket: its distinct keys (or kOver).
template <typename K>
__global__ __launch_bounds__(kLongThreads) void k_big_scan(const uint32_t* __restrict__ offsets,
                                                           const K* __restrict__ keys, BigWork<K> bw) {
  constexpr int W = kLongThreads / kWave;
  __shared__ K sval[W][kSetMax];
  __shared__ uint32_t scnt[W][kSetMax];
  __shared__ uint32_t ssize[W];
  __shared__ uint32_t soverflow;
  const uint32_t t = threadIdx.x;
  const uint32_t nch = bw.ctr[1];
  for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const uint32_t g = bw.big_g[bw.chunk_b[c]];
    const uint32_t lo = offsets[g], L = offsets[g + 1] - lo;
    const uint32_t a = bw.chunk_k[c] * kBigChunk, b = min(L, a + kBigChunk);
    wg_distinct<K, kLongThreads>(keys + lo, a, b, sval, scnt, ssize, &soverflow);
    const uint32_t nd = wave_uniform(soverflow) ? kOver : wave_uniform(ssize[0]);
    if (t == 0) bw.chunk_n[c] = nd;
    if (nd != kOver && t < nd) {
      bw.chunk_key[static_cast<size_t>(c) * kSetMax + t] = sval[0][t];
      bw.chunk_cnt[static_cast<size_t>(c) * kSetMax + t] = scnt[0][t];
    }
    __syncthreads();
  }
}

// One workgroup per big bucket: the chunk sets merged, ranked into runs;
// too many distinct keys list the bucket as unsorted.  Wave w merges chunks
// w, w + W, ... into its own set, then wave 0 merges the W sets (a bucket of
// one heavy key has one chunk per 2^16 of its copies).
template <typename K>
__global__ __launch_bounds__(kLongThreads) void k_big_fix(const uint32_t* __restrict__ offsets, BigWork<K> bw,
                                                          uint32_t* __restrict__ unsorted) {
  constexpr int W = kLongThreads / kWave;
  __shared__ K sval[W][kSetMax];
  __shared__ uint32_t scnt[W][kSetMax];
  __shared__ uint32_t ssize[W];
  __shared__ uint32_t run0[kSetMax + 1];
  __shared__ uint32_t soverflow;
  const uint32_t t = threadIdx.x, w = t / kWave, l = lane_id();
  const uint32_t nbig = bw.ctr[0];
  for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    const uint32_t g = bw.big_g[bi];
    const uint32_t L = offsets[g + 1] - offsets[g];
    const uint32_t first = bw.big_first[bi], nch = (L + kBigChunk - 1) / kBigChunk;
    if (t < W) ssize[t] = 0;
    if (t == 0) soverflow = 0;
    __syncthreads();
    {
      bool full = false;
      for (uint32_t c = first + w; c < first + nch && !full; c += W) {
        const uint32_t nd = wave_uniform(bw.chunk_n[c]);
        if (nd == kOver) {
          if (l == 0) soverflow = 1;
          break;
        }
        for (uint32_t e = 0; e < nd; ++e) {
          if (!set_add(sval[w], scnt[w], &ssize[w], bw.chunk_key[static_cast<size_t>(c) * kSetMax + e],
                       bw.chunk_cnt[static_cast<size_t>(c) * kSetMax + e])) {
            if (l == 0) soverflow = 1;
            full = true;
            break;
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    if (w == 0 && wave_uniform(soverflow) == 0) {
      bool full = false;
      for (uint32_t o = 1; o < static_cast<uint32_t>(W) && !full; ++o) {
        const uint32_t n = wave_uniform(ssize[o]);
        for (uint32_t e = 0; e < n; ++e) {
          if (!set_add(sval[0], scnt[0], &ssize[0], sval[o][e], scnt[o][e])) {
            if (l == 0) soverflow = 1;
            full = true;
            break;
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    if (wave_uniform(soverflow)) {
      if (t == 0) {
        bw.run_n[bi] = kOver;
        const uint32_t u = atomicAdd(&unsorted[0], 1u);
        if (u < kMaxUnsorted) unsorted[1 + u] = g;
      }
    } else {
      const uint32_t nd = wave_uniform(ssize[0]);
      rank_runs<K>(nd, sval, scnt, run0);
      if (t < nd) bw.run_key[static_cast<size_t>(bi) * kSetMax + t] = sval[1][t];
      if (t <= nd) bw.run0[static_cast<size_t>(bi) * (kSetMax + 1) + t] = run0[t];
      if (t == 0) bw.run_n[bi] = nd;
    }
    __syncthreads();
  }
}

// Every chunk of a big bucket with 2 .. kSetMax distinct keys: its range
// rewritten from the bucket's runs.
template <typename K>
__global__ __launch_bounds__(kLongThreads) void k_big_write(const uint32_t* __restrict__ offsets,
                                                            K* __restrict__ keys, BigWork<K> bw) {
  __shared__ uint32_t run0[kSetMax + 1];
  __shared__ K rkey[kSetMax];
  const uint32_t t = threadIdx.x;
  const uint32_t nch = bw.ctr[1];
  for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const uint32_t bi = bw.chunk_b[c];
    const uint32_t nd = bw.run_n[bi];
    if (nd == kOver || nd <= 1) continue;  // uniform over the workgroup
    const uint32_t g = bw.big_g[bi];
    const uint32_t lo = offsets[g], L = offsets[g + 1] - lo;
    const uint32_t a = bw.chunk_k[c] * kBigChunk, b = min(L, a + kBigChunk);
    __syncthreads();  // the previous chunk is done with run0 / rkey
    if (t <= nd) run0[t] = bw.run0[static_cast<size_t>(bi) * (kSetMax + 1) + t];
    if (t < nd) rkey[t] = bw.run_key[static_cast<size_t>(bi) * kSetMax + t];
    __syncthreads();
    uint32_t r = 0;
    for (uint32_t i = a + t; i < b; i += kLongThreads) {
      while (r + 1 < nd && run0[r + 1] <= i) ++r;
      keys[lo + i] = rkey[r];
    }
  }
}

__global__ __launch_bounds__(256) void k_find_long(const uint32_t* __restrict__ offsets,
                                                   const uint32_t* __restrict__ nb, uint32_t* __restrict__ long_count,
                                                   uint32_t* __restrict__ long_list) {
  const uint32_t B = *nb;
  for (uint32_t g = blockIdx.x * 256u + threadIdx.x; g < B; g += gridDim.x * 256u)
    if (offsets[g + 1] - offsets[g] > kLongT) note_long(long_count, long_list, g, offsets[g + 1] - offsets[g]);
}

template <typename K, int THREADS, int ITEMS, int MAXD, int OP>
hipError_t msplit_dig(int dig, dim3 grid, const K* in, uint32_t n, const SegPlan* plan, uint32_t nd, uint32_t log2P,
                      uint32_t P, const PartDesc* desc, uint32_t shift, uint32_t* counts, K* out, uint16_t* perm,
                      hipStream_t s) {
  if (dig == DIG_RANGE) {
    if constexpr (MAXD <= 256) {  // level 1 only
      k_msplit<K, THREADS, ITEMS, MAXD, OP, DIG_RANGE><<<grid, THREADS, 0, s>>>(in, n, plan, nd, log2P, P, desc,
                                                                               shift, counts, out, perm);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (dig == DIG_PART)
    k_msplit<K, THREADS, ITEMS, MAXD, OP, DIG_PART><<<grid, THREADS, 0, s>>>(in, n, plan, nd, log2P, P, desc, shift,
                                                                            counts, out, perm);
  else if (dig == DIG_COARSE)
    k_msplit<K, THREADS, ITEMS, MAXD, OP, DIG_COARSE><<<grid, THREADS, 0, s>>>(in, n, plan, nd, log2P, P, desc, shift,
                                                                              counts, out, perm);
  else
    k_msplit<K, THREADS, ITEMS, MAXD, OP, DIG_SUB><<<grid, THREADS, 0, s>>>(in, n, plan, nd, log2P, P, desc, shift,
                                                                           counts, out, perm);
  return hipGetLastError();
}

template <typename K, int THREADS, int ITEMS, int MAXD>
hipError_t msplit_op(int op, int dig, dim3 grid, const K* in, uint32_t n, const SegPlan* plan, uint32_t nd,
                     uint32_t log2P, uint32_t P, const PartDesc* desc, uint32_t shift, uint32_t* counts, K* out,
                     uint16_t* perm, hipStream_t s) {
  if (op == OP_COUNT)
    return msplit_dig<K, THREADS, ITEMS, MAXD, OP_COUNT>(dig, grid, in, n, plan, nd, log2P, P, desc, shift, counts,
                                                        out, perm, s);
  return msplit_dig<K, THREADS, ITEMS, MAXD, OP_SCATTER>(dig, grid, in, n, plan, nd, log2P, P, desc, shift, counts,
                                                        out, perm, s);
}

template <typename K>
hipError_t msplit_level(int level, int op, int dig, const K* in, uint32_t n, uint32_t max_tiles, const SegPlan* plan,
                        uint32_t nd, uint32_t log2P, uint32_t P, const PartDesc* desc, uint32_t shift,
                        uint32_t* counts, K* out, uint16_t* perm, hipStream_t s) {
  if (level == 1) {
    const uint32_t tiles = div_up(n, kL1Tile);
    if (tiles == 0) return hipSuccess;
    if (nd > 256) return hipErrorInvalidValue;
    return msplit_op<K, kL1Threads, kL1Items, 256>(op, dig, dim3(tiles), in, n, nullptr, nd, log2P, P, desc, shift, counts,
                                              out, perm, s);
  }
  if (max_tiles == 0) return hipSuccess;
  // Both passes cut the same tiles (kL2Threads * kItems2 keys); counting
  // runs them with half the threads and twice the items.
  constexpr int kItems2 = sizeof(K) == 4 ? 8 : 4;
  if (op == OP_COUNT)
    return msplit_op<K, kL2Threads / 2, 2 * kItems2, kMaxD2>(op, dig, dim3(max_tiles), in, n, plan, nd, log2P, P,
                                                              desc, shift, counts, out, perm, s);
  return msplit_op<K, kL2Threads, kItems2, kMaxD2>(op, dig, dim3(max_tiles), in, n, plan, nd, log2P, P, desc, shift,
                                                    counts, out, perm, s);
}

}  // namespace

hipError_t launch_msplit(int kt, int level, int op, int dig, const void* in, uint32_t n, uint32_t max_tiles,
                         const SegPlan* plan, uint32_t nd, uint32_t log2P, uint32_t P, const PartDesc* desc,
                         uint32_t shift, uint32_t* counts, void* out, uint16_t* perm, hipStream_t s) {
  if (kt == 0)
    return msplit_level<uint32_t>(level, op, dig, static_cast<const uint32_t*>(in), n, max_tiles, plan, nd, log2P, P,
                                  desc, shift, counts, static_cast<uint32_t*>(out), perm, s);
  return msplit_level<uint64_t>(level, op, dig, static_cast<const uint64_t*>(in), n, max_tiles, plan, nd, log2P, P,
                                desc, shift, counts, static_cast<uint64_t*>(out), perm, s);
}

template <int THREADS, int ITEMS, int MAXD, int SB>
hipError_t tile_gather_sb(dim3 grid, const uint16_t* perm, const void* src, uint32_t n, const SegPlan* plan,
                          uint32_t nd, const uint32_t* scan, const uint32_t* unsorted, void* out, int out_kind,
                          hipStream_t s) {
  if (out_kind == GATHER_FOUND)
    k_tile_gather<THREADS, ITEMS, MAXD, GATHER_FOUND, SB><<<grid, THREADS, 0, s>>>(perm, src, n, plan, nd, scan,
                                                                                  unsorted, out);
  else if (out_kind == GATHER_COUNT)
    k_tile_gather<THREADS, ITEMS, MAXD, GATHER_COUNT, SB><<<grid, THREADS, 0, s>>>(perm, src, n, plan, nd, scan,
                                                                                  unsorted, out);
  else
    k_tile_gather<THREADS, ITEMS, MAXD, GATHER_STAGE, SB><<<grid, THREADS, 0, s>>>(perm, src, n, plan, nd, scan,
                                                                                  unsorted, out);
  return hipGetLastError();
}

// Byte counts first (no long bucket, the common case), then word counts;
// exactly one of the two does the work (the table's flag decides on the
// device, so nothing waits for the host).
template <int THREADS, int ITEMS, int MAXD>
hipError_t tile_gather(dim3 grid, const uint16_t* perm, const void* src, uint32_t n, const SegPlan* plan,
                       uint32_t nd, const uint32_t* scan, const uint32_t* unsorted, void* out, int out_kind,
                       hipStream_t s) {
  hipError_t e = tile_gather_sb<THREADS, ITEMS, MAXD, 1>(grid, perm, src, n, plan, nd, scan, unsorted, out,
                                                         out_kind, s);
  if (e != hipSuccess) return e;
  return tile_gather_sb<THREADS, ITEMS, MAXD, 4>(grid, perm, src, n, plan, nd, scan, unsorted, out, out_kind, s);
}

hipError_t launch_tile_gather(int kt, int level, const uint16_t* perm, const void* src, uint32_t n,
                              uint32_t max_tiles, const SegPlan* plan, uint32_t nd, const uint32_t* scan,
                              const uint32_t* unsorted, void* out, int out_kind, hipStream_t s) {
  if (level == 1) {
    const uint32_t tiles = div_up(n, kL1Tile);
    if (tiles == 0) return hipSuccess;
    if (nd > 256) return hipErrorInvalidValue;
    return tile_gather<kL1Tile / 16, 16, 256>(dim3(tiles), perm, src, n, nullptr, nd, scan, unsorted, out,
                                              out_kind, s);
  }
  if (max_tiles == 0) return hipSuccess;
  // Half the split's threads, twice the items: a tile's gather takes eight
  // waves, so four of them fit on a CU instead of two.
  if (kt == 0)
    return tile_gather<kL2Threads / 2, 16, kMaxD2>(dim3(max_tiles), perm, src, n, plan, 0, scan, unsorted, out,
                                                   out_kind, s);
  return tile_gather<kL2Threads / 2, 8, kMaxD2>(dim3(max_tiles), perm, src, n, plan, 0, scan, unsorted, out,
                                                out_kind, s);
}

hipError_t launch_plan(const uint32_t* scan1, uint32_t tiles1, uint32_t nseg, uint32_t n, int mode,
                       const uint32_t* bucket_base, const uint32_t* nb_total, const uint32_t* seg_keys, uint32_t sh1,
                       uint32_t log2S, uint32_t tile2, uint32_t max_tiles, uint32_t max_subbins, uint32_t* offsets,
                       SegPlan* plan, hipStream_t s) {
  k_plan<<<1, kPlanThreads, 0, s>>>(scan1, tiles1, nseg, n, mode, bucket_base, nb_total, seg_keys, sh1, log2S, tile2,
                                    max_tiles, max_subbins, offsets, plan);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t m = max_tiles > max_subbins ? max_tiles : max_subbins;
  if (m > 0) k_seg_map<<<div_up(m, 256), 256, 0, s>>>(plan);
  return hipGetLastError();
}

hipError_t launch_batch_layout(const uint32_t* table_keys, uint32_t T, uint32_t n, uint32_t num, uint32_t den,
                               uint32_t* part_offsets, uint32_t* bucket_base, PartDesc* desc, hipStream_t s) {
  k_batch_layout<<<1, kPlanThreads, 0, s>>>(table_keys, T, n, num, den, part_offsets, bucket_base, desc);
  return hipGetLastError();
}

uint32_t heavy_chunk_keys() { return kHeavyChunk; }

template <typename K>
hipError_t lds_build_passes(const K* in, const SegPlan* plan, const uint32_t* scan2, uint32_t max_subbins,
                            uint32_t log2P, uint32_t P, const PartDesc* desc, uint32_t* offsets, K* out,
                            uint32_t* long_count, uint32_t* long_list, uint32_t* heavy, uint32_t max_chunks,
                            uint32_t* long_flags, hipStream_t s) {
  // 64-bit keys: 105 VGPRs, four waves per SIMD.  (1024 threads x 10 keys
  // at eight waves per SIMD spills across the scan and measured slower.)
  constexpr int kMinW = sizeof(K) == 4 ? 8 : 4;
  uint32_t* heavy_chunks = heavy + 2;
  uint32_t* heavy_bins = heavy_chunks + 2 * static_cast<size_t>(max_chunks);
  hipError_t e = launch_fill_u32(heavy, 2, 0u, s);
  if (e != hipSuccess) return e;
  if constexpr (sizeof(K) == 4) {
    if ((e = launch_fill_u32(long_flags, max_subbins, 0u, s)) != hipSuccess) return e;
  }
  k_lds_build<K, kBuildThreads, 20, kMinW><<<max_subbins, kBuildThreads, 0, s>>>(
      in, plan, scan2, log2P, P, desc, offsets, out, long_count, long_list, heavy, heavy_chunks, heavy_bins,
      long_flags);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if constexpr (sizeof(K) == 4) {
    constexpr uint32_t kNoteGrid = 1024;
    k_note_long<kBuildThreads><<<max_subbins < kNoteGrid ? max_subbins : kNoteGrid, kBuildThreads, 0, s>>>(
        plan, scan2, offsets, long_flags, long_count, long_list);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  constexpr uint32_t kGrid = 1024, kBinGrid = 256;
  k_heavy_count<K, kBuildThreads, 20><<<kGrid, kBuildThreads, 0, s>>>(in, plan, scan2, log2P, P, desc, offsets,
                                                                      heavy, heavy_chunks);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_heavy_scan<kBuildThreads><<<kBinGrid, kBuildThreads, 0, s>>>(plan, scan2, offsets, heavy, heavy_bins);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_heavy_scatter<K, kBuildThreads, 20><<<kGrid, kBuildThreads, 0, s>>>(in, plan, scan2, log2P, P, desc, offsets,
                                                                        out, heavy, heavy_chunks);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_heavy_fix<kBuildThreads><<<kBinGrid, kBuildThreads, 0, s>>>(plan, scan2, offsets, heavy, heavy_bins, long_count,
                                                                long_list);
  return hipGetLastError();
}

hipError_t launch_lds_build(int kt, const void* in, const SegPlan* plan, const uint32_t* scan2, uint32_t max_subbins,
                            uint32_t log2P, uint32_t P, const PartDesc* desc, uint32_t* offsets, void* out,
                            uint32_t* long_count, uint32_t* long_list, uint32_t* heavy, uint32_t max_chunks,
                            uint32_t* long_flags, hipStream_t s) {
  if (max_subbins == 0) return hipSuccess;
  if (kt == 0)
    return lds_build_passes(static_cast<const uint32_t*>(in), plan, scan2, max_subbins, log2P, P, desc, offsets,
                            static_cast<uint32_t*>(out), long_count, long_list, heavy, max_chunks, long_flags, s);
  return lds_build_passes(static_cast<const uint64_t*>(in), plan, scan2, max_subbins, log2P, P, desc, offsets,
                          static_cast<uint64_t*>(out), long_count, long_list, heavy, max_chunks, long_flags, s);
}

uint32_t probe_chunk_keys(int kt) { return kLdsThreads * (kt == 0 ? kProbeReg32 : kProbeReg64); }

hipError_t launch_lds_probe(int kt, const void* q2, const SegPlan* qplan, const uint32_t* qscan2,
                            uint32_t max_subbins, uint32_t q, uint32_t log2P, uint32_t P, const PartDesc* desc,
                            const uint32_t* offsets, const void* tkeys, const uint32_t* unsorted, uint32_t log2W,
                            uint32_t* queue, void* c2, hipStream_t s) {
  if (max_subbins == 0) return hipSuccess;
  const uint32_t ch = probe_chunk_keys(kt);
  const uint32_t max_queued = q / ch + 1;
  hipError_t e = launch_fill_u32(queue, 1, 0u, s);
  if (e != hipSuccess) return e;
  k_probe_queue<<<div_up(max_subbins, 256), 256, 0, s>>>(qplan, qscan2, ch, queue);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint32_t grid = max_subbins + max_queued;
  if (kt == 0)
    k_lds_probe<uint32_t, kLdsThreads, kProbeReg32, 8><<<grid, kLdsThreads, 0, s>>>(
        static_cast<const uint32_t*>(q2), qplan, qscan2, log2P, P, desc, offsets, static_cast<const uint32_t*>(tkeys),
        unsorted, log2W, queue, max_queued, c2);
  else
    k_lds_probe<uint64_t, kLdsThreads, kProbeReg64, 8><<<grid, kLdsThreads, 0, s>>>(
        static_cast<const uint64_t*>(q2), qplan, qscan2, log2P, P, desc, offsets, static_cast<const uint64_t*>(tkeys),
        unsorted, log2W, queue, max_queued, c2);
  return hipGetLastError();
}

hipError_t launch_find_long(const uint32_t* offsets, const uint32_t* num_buckets_dev, uint64_t bound,
                            uint32_t* long_count, uint32_t* long_list, hipStream_t s) {
  if (bound == 0) return hipSuccess;
  const uint64_t blocks = (bound + 255) / 256;
  k_find_long<<<static_cast<uint32_t>(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(offsets, num_buckets_dev,
                                                                                   long_count, long_list);
  return hipGetLastError();
}

template <typename K>
hipError_t long_sort_typed(const uint32_t* offsets, uint32_t* ctr, uint32_t* list, K* keys, uint32_t* unsorted,
                           uint32_t* big, uint64_t n, hipStream_t s) {
  const BigWork<K> bw = big_work<K>(big, n);
  hipError_t e = launch_fill_u32(bw.ctr, 2, 0u, s);
  if (e != hipSuccess) return e;
  k_long_small<K, kLongThreads, false><<<kLongGrid, kLongThreads, 0, s>>>(offsets, ctr, list, keys, unsorted);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_long_small<K, kLongWaveThreads, true>
      <<<kLongGrid * (kLongThreads / kLongWaveThreads), kLongWaveThreads, 0, s>>>(offsets, ctr, list, keys, unsorted);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_long_sort<K><<<kLongGrid, kLongThreads, 0, s>>>(offsets, ctr, list, keys, unsorted, bw);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_long_wgsort<K><<<kLongGrid, kLongThreads, 0, s>>>(offsets, ctr, list, keys);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_big_scan<K><<<kLongGrid, kLongThreads, 0, s>>>(offsets, keys, bw);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_big_fix<K><<<kLongGrid / 2, kLongThreads, 0, s>>>(offsets, bw, unsorted);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_big_write<K><<<kLongGrid, kLongThreads, 0, s>>>(offsets, keys, bw);
  return hipGetLastError();
}

hipError_t launch_long_sort(int kt, const uint32_t* offsets, uint32_t* long_ctr, uint32_t* long_list, void* keys,
                            uint32_t* unsorted, uint32_t* big, uint64_t n, hipStream_t s) {
  if (kt == 0)
    return long_sort_typed<uint32_t>(offsets, long_ctr, long_list, static_cast<uint32_t*>(keys), unsorted, big, n,
                                     s);
  return long_sort_typed<uint64_t>(offsets, long_ctr, long_list, static_cast<uint64_t*>(keys), unsorted, big, n, s);
}

}  // namespace hg
