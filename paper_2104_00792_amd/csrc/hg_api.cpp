// C ABI of the HashGraph library: argument validation, memory, launch order.
//
// Every argument check happens before the first HIP call, so the error paths
// run on machines without a GPU.  Device memory comes from a stream-ordered
// pool owned by the library (one per device, never trimmed), so repeated
// builds do not reach the driver's allocator and nothing synchronizes.
#include "hg.h"

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hg_internal.h"

// Caller-supplied device allocator (hg_set_allocator); empty = the pool.
struct AllocHook {
  hg_alloc_fn alloc = nullptr;
  hg_free_fn free_fn = nullptr;
  void* ctx = nullptr;
};

// A device block and the allocator it goes back to.
struct TableBlock {
  void* p;
  size_t bytes;
  AllocHook hook;
};

struct hg_table {
  int device;
  hipStream_t stream;
  hg_key_type kt;
  uint64_t n;
  uint32_t P;
  uint32_t log2P;
  uint64_t buckets_bound;   // upper bound of sum(V_p) used for the allocation
  void* d_keys;             // n keys, bucket-contiguous
  uint32_t* d_offsets;      // buckets_bound + 1
  void* d_meta;             // part_offsets | bucket_base | desc
  uint32_t* d_part_offsets; // P + 1
  uint32_t* d_bucket_base;  // P + 1
  hg::PartDesc* d_desc;     // P
  uint32_t* d_unsorted;     // kUnsortedWords: long buckets left unsorted, has-long word
  int split_mode;           // level-1 split: 0 by partition, 1 by coarse bucket range
  uint32_t sh1;             // coarse range 2^sh1 buckets (mode 1)
  uint32_t nd1;             // level-1 digits
  uint32_t log2S;           // sub-bins of 2^log2S buckets
  bool batched;             // P caller-defined tables (hg_build_batched)
  uint64_t id;              // nonzero, unique in the process
  uint64_t like_id;         // id of the table whose layout this one copies (hg_build_like), else 0
  std::vector<TableBlock> blocks;  // keys, offsets and metadata, and where they go back
  std::mutex mu;
  bool have_num_buckets;
  uint64_t num_buckets;
  uint32_t has_long;  // read with num_buckets
};

namespace {

thread_local std::string t_err;

hg_status fail(hg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_err = buf;
  return s;
}

hg_status fail_hip(hipError_t e, const char* where) {
  return fail(e == hipErrorOutOfMemory ? HG_ERR_OUT_OF_MEMORY : HG_ERR_HIP, "%s: %s", where,
              hipGetErrorString(e));
}

bool debug_sync() {
  static const bool on = [] {
    const char* v = std::getenv("HG_DEBUG_SYNC");
    return v != nullptr && v[0] != '\0' && v[0] != '0';
  }();
  return on;
}

// ------------------------------------------------------------ block cache
// The library's own device memory: blocks from hipMalloc that stay cached
// after they are freed.  A block freed on stream s serves later requests on
// s at once (stream order keeps its last use ahead of the next), and
// requests on other streams once the event recorded at its free has
// completed.  In the steady state of repeated calls nothing here waits for
// the device, so a caller can enqueue call after call while the GPU works
// (a stream-ordered hipMemPool has been measured to block the host in
// every allocation that reuses a block).  Only hipMalloc of a new block,
// the out-of-memory path and hg_trim_pool wait.
struct CachedBlock {
  void* p;
  size_t bytes;     // rounded size
  hipStream_t s;    // stream of its last use
  hipEvent_t ev;    // recorded on s at its free
};
struct DevCache {
  std::multimap<size_t, CachedBlock> idle;  // by rounded size
  std::vector<hipEvent_t> events;           // recorded events no block holds
  uint64_t idle_bytes = 0;
};
struct LiveBlock {
  int dev;
  size_t bytes;
};
std::mutex g_cache_mu;
std::map<int, DevCache> g_cache;
std::map<void*, LiveBlock> g_live;

// Sizes are rounded so that blocks of nearly equal requests are shared:
// 512 bytes up to 1 MiB, 2 MiB above.  A request takes an idle block of its
// rounded size up to an eighth more.
size_t cache_round(size_t b) {
  const size_t g = b <= (size_t(1) << 20) ? 512 : (size_t(2) << 20);
  return (b + g - 1) / g * g;
}

// Hands idle blocks of dev back to HIP, largest first, until at most keep
// bytes stay idle; waits for each block's last use.  Caller holds the lock
// with dev current.
hipError_t cache_release(DevCache& c, uint64_t keep) {
  hipError_t first = hipSuccess;
  while (c.idle_bytes > keep && !c.idle.empty()) {
    auto it = std::prev(c.idle.end());
    const CachedBlock b = it->second;
    c.idle.erase(it);
    c.idle_bytes -= b.bytes;
    hipError_t e = hipEventSynchronize(b.ev);
    if (e == hipSuccess) e = hipFree(b.p);
    if (e != hipSuccess && first == hipSuccess) first = e;
    c.events.push_back(b.ev);
  }
  return first;
}

hipError_t cache_alloc(int dev, void** p, size_t bytes, hipStream_t s) {
  const size_t r = cache_round(bytes);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  DevCache& c = g_cache[dev];
  auto pick = c.idle.end();
  for (auto it = c.idle.lower_bound(r); it != c.idle.end() && it->first <= r + r / 8; ++it) {
    if (it->second.s == s) {
      pick = it;
      break;
    }
    if (pick == c.idle.end()) {
      const hipError_t q = hipEventQuery(it->second.ev);
      if (q == hipSuccess)
        pick = it;
      else
        (void)hipGetLastError();  // not ready: no error for the caller's later checks
    }
  }
  if (pick != c.idle.end()) {
    *p = pick->second.p;
    c.events.push_back(pick->second.ev);
    c.idle_bytes -= pick->second.bytes;
    g_live[*p] = {dev, pick->second.bytes};
    c.idle.erase(pick);
    return hipSuccess;
  }
  hipError_t e = hipMalloc(p, r);
  if (e == hipErrorOutOfMemory) {
    // Idle blocks of other sizes hold the memory: give them back, once.
    (void)hipGetLastError();
    (void)cache_release(c, 0);
    e = hipMalloc(p, r);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  g_live[*p] = {dev, r};
  return hipSuccess;
}

// Takes back a block in stream order: work enqueued on s before this call
// may still use it.
void cache_free(void* p, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) return;
  const LiveBlock lb = it->second;
  g_live.erase(it);
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != lb.dev) (void)hipSetDevice(lb.dev);
  DevCache& c = g_cache[lb.dev];
  hipEvent_t ev = nullptr;
  if (!c.events.empty()) {
    ev = c.events.back();
    c.events.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    ev = nullptr;
  }
  if (ev != nullptr && hipEventRecord(ev, s) == hipSuccess) {
    c.idle.emplace(lb.bytes, CachedBlock{p, lb.bytes, s, ev});
    c.idle_bytes += lb.bytes;
  } else {
    // No event to order its reuse: wait for the stream and give it back.
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    (void)hipFree(p);
    if (ev != nullptr) c.events.push_back(ev);
  }
  if (cur >= 0 && cur != lb.dev) (void)hipSetDevice(cur);
}

std::atomic<uint64_t> g_next_table_id{1};

// ------------------------------------------------------- allocator hook
std::mutex g_hook_mu;
AllocHook g_hook;

AllocHook current_hook() {
  std::lock_guard<std::mutex> lk(g_hook_mu);
  return g_hook;
}

// Dry run of one call (hg_workspace_size): blocks are counted and handed out
// as addresses that are never dereferenced on the host, and nothing reaches
// the device.
struct Measure {
  uint64_t workspace = 0;
  uint64_t table = 0;
  uintptr_t next = uintptr_t(1) << 44;
};
thread_local Measure* t_measure = nullptr;

uint64_t round256(uint64_t b) { return (b + 255) & ~uint64_t(255); }

hipError_t current_device(int* dev) {
  if (t_measure) {
    *dev = 0;
    return hipSuccess;
  }
  return hipGetDevice(dev);
}

void free_block(const TableBlock& b, hipStream_t s) {
  if (b.p == nullptr || t_measure) return;
  if (b.hook.free_fn)
    b.hook.free_fn(b.p, b.bytes, s, b.hook.ctx);
  else
    cache_free(b.p, s);
}

// Outcome of one allocation: a HIP status, or a block from the caller's
// allocator that breaks its alignment contract.
struct AllocResult {
  hipError_t e;
  bool misaligned;
};

// Allocations of one call; frees everything still owned on destruction.
class Allocs {
 public:
  explicit Allocs(hipStream_t s) : s_(s), hook_(current_hook()) {}
  ~Allocs() {
    for (const TableBlock& b : owned_) free_block(b, s_);
  }
  AllocResult get(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return {hipSuccess, false};
    if (t_measure) {
      const uint64_t r = round256(bytes);
      *p = reinterpret_cast<void*>(t_measure->next);
      t_measure->next += r;
      t_measure->workspace += r;
      owned_.push_back({*p, bytes, hook_});
      return {hipSuccess, false};
    }
    if (hook_.alloc) {
      *p = hook_.alloc(bytes, s_, hook_.ctx);
      if (*p == nullptr) return {hipErrorOutOfMemory, false};
      if (reinterpret_cast<uintptr_t>(*p) & 255u) {
        hook_.free_fn(*p, bytes, s_, hook_.ctx);
        *p = nullptr;
        return {hipSuccess, true};
      }
      owned_.push_back({*p, bytes, hook_});
      return {hipSuccess, false};
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return {e, false};
    e = cache_alloc(dev, p, bytes, s_);
    if (e == hipSuccess) owned_.push_back({*p, bytes, hook_});
    return {e, false};
  }
  // Stop owning p: it now belongs to a table.
  TableBlock release(void* p) {
    TableBlock out{nullptr, 0, hook_};
    std::vector<TableBlock> keep;
    for (const TableBlock& b : owned_) {
      if (b.p == p && p != nullptr)
        out = b;
      else
        keep.push_back(b);
    }
    owned_.swap(keep);
    if (t_measure && out.p) {
      t_measure->workspace -= round256(out.bytes);
      t_measure->table += round256(out.bytes);
    }
    return out;
  }

 private:
  hipStream_t s_;
  AllocHook hook_;
  std::vector<TableBlock> owned_;
};

// -------------------------------------------------------------- profiling
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::string g_prof_only;  // empty: every launch
std::vector<ProfRec> g_pending;
std::vector<hipEvent_t> g_events;
std::map<std::string, std::pair<uint64_t, double>> g_totals;

hipEvent_t take_event() {
  if (!g_events.empty()) {
    hipEvent_t e = g_events.back();
    g_events.pop_back();
    return e;
  }
  // Timing only: a device-scope release keeps the record from writing back
  // and invalidating the caches between the bracketed kernels.
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t s) : name_(name), s_(s) {
    if (t_measure) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || (!g_prof_only.empty() && g_prof_only != name_)) return;
    a_ = take_event();
    b_ = take_event();
    if (a_ && b_) (void)hipEventRecord(a_, s_);
  }
  ~ProfScope() {
    if (!a_ || !b_) return;
    (void)hipEventRecord(b_, s_);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_pending.push_back({name_, a_, b_});
  }

 private:
  const char* name_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

#define HG_LAUNCH(name, stream, call)                                       \
  do {                                                                      \
    hipError_t _e;                                                          \
    {                                                                       \
      ProfScope _ps(name, stream);                                          \
      _e = t_measure ? hipSuccess : (call);                                 \
    }                                                                       \
    if (_e != hipSuccess) return fail_hip(_e, name);                        \
    if (debug_sync() && !t_measure) {                                       \
      _e = hipStreamSynchronize(stream);                                    \
      std::fprintf(stderr, "[hg] %s -> %s\n", name, hipGetErrorString(_e)); \
      if (_e != hipSuccess) return fail_hip(_e, name);                      \
    }                                                                       \
  } while (0)

hg_status to_status(hipError_t e, const char* what) { return e == hipSuccess ? HG_OK : fail_hip(e, what); }

hg_status to_status(AllocResult r, const char* what) {
  if (r.misaligned) return fail(HG_ERR_INVALID_ARG, "%s: the allocator returned a block not aligned to 256 bytes", what);
  return to_status(r.e, what);
}

#define HG_TRY(expr, what)                      \
  do {                                          \
    hg_status _s = to_status((expr), what);     \
    if (_s != HG_OK) return _s;                 \
  } while (0)

uint32_t log2_of(uint32_t P) {
  uint32_t l = 0;
  while ((1u << l) < P) ++l;
  return l;
}

bool is_pow2(uint32_t x) { return x != 0 && (x & (x - 1)) == 0; }

size_t key_bytes(hg_key_type kt) { return kt == HG_KEY_U32 ? 4 : 8; }

hg_status check_n_P(uint64_t n, hg_key_type kt, uint32_t P) {
  if (kt != HG_KEY_U32 && kt != HG_KEY_U64) return fail(HG_ERR_INVALID_ARG, "unknown key type %d", (int)kt);
  if (n >= (1ull << 32)) return fail(HG_ERR_INVALID_ARG, "n = %llu is not below 2^32", (unsigned long long)n);
  if (!is_pow2(P)) return fail(HG_ERR_INVALID_ARG, "P = %u is not a power of two", P);
  if (P > hg::kMaxP) return fail(HG_ERR_UNSUPPORTED, "P = %u exceeds %u", P, hg::kMaxP);
  return HG_OK;
}

// Partition split of n keys into `out` (a2-a4).  tile_counts must hold
// P * num_tiles words, bsums the scan's block sums.
hg_status run_partition(const void* keys, uint32_t n, hg_key_type kt, uint32_t log2P, uint32_t num_tiles,
                        uint32_t* tile_counts, uint32_t* bsums, void* out, hipStream_t s) {
  const uint32_t P = 1u << log2P;
  HG_LAUNCH("part_count", s, hg::launch_part_count(kt, keys, n, log2P, num_tiles, tile_counts, s));
  HG_LAUNCH("part_scan", s,
            hg::launch_scan_exclusive(tile_counts, nullptr, static_cast<uint64_t>(P) * num_tiles, bsums, s));
  HG_LAUNCH("part_scatter", s, hg::launch_part_scatter(kt, keys, n, log2P, num_tiles, tile_counts, out, s));
  return HG_OK;
}


// ------------------------------------------------ level-1 split parameters
uint32_t ceil_log2(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

// Workspace of the heavy sub-bin passes for n keys (see launch_lds_build).
struct HeavyWork {
  uint32_t* words = nullptr;
  uint32_t max_chunks = 0;
  uint32_t* long_flags = nullptr;  // one word per sub-bin
};

hg_status alloc_heavy(Allocs& mem, uint64_t n, uint32_t max_subbins, HeavyWork& h) {
  const uint64_t max_heavy = n / 65536 + 1;
  const uint64_t max_chunks = n / hg::heavy_chunk_keys() + max_heavy + 1;
  const uint64_t heavy_words = 2 + 2 * max_chunks + max_heavy;
  void* p = nullptr;
  HG_TRY(mem.get(&p, (heavy_words + std::max<uint64_t>(max_subbins, 1)) * sizeof(uint32_t)),
         "allocate heavy sub-bin queue");
  h.words = static_cast<uint32_t*>(p);
  h.max_chunks = static_cast<uint32_t>(max_chunks);
  h.long_flags = h.words + heavy_words;
  return HG_OK;
}

// Level-2 tiles of n keys in nseg segments: a segment of n_s keys whose
// tiles start up to kTileAlign - 1 keys early has at most
// (n_s + kTileAlign - 2) / tile + 1 of them.
uint32_t max_l2_tiles(uint64_t n, uint32_t tile, uint32_t nseg) {
  return hg::div_up(n + static_cast<uint64_t>(hg::kTileAlign - 2) * nseg, tile) + nseg;
}

struct SplitParams {
  int mode;        // 0: partitions, 1: coarse bucket ranges
  uint32_t sh1;    // mode 1: 2^sh1 buckets per range
  uint32_t nd1;    // level-1 digits
  uint32_t log2S;  // regular sub-bins hold 2^log2S buckets
};

// Level-2 digits per segment: at most 2^L2 (L2 in 7..10, HG_SPLIT_L2_BITS,
// default 8).  Fewer level-2 digits make the level-2 ranking cheaper and its
// runs longer at the price of more level-1 digits.
uint32_t split_l2_bits() {
  static const uint32_t bits = [] {
    const char* v = std::getenv("HG_SPLIT_L2_BITS");
    const long b = v ? std::strtol(v, nullptr, 10) : 8;
    return static_cast<uint32_t>(b < 7 ? 7 : (b > 10 ? 10 : b));
  }();
  return bits;
}

// Sub-bins of about 2^13 keys (log2S shrinks as keys per bucket grow).
// Level-1 digits by partition when an average partition's table fits 2^L2
// sub-bins (the last of which may grow to 2^kLog2SLds buckets in LDS);
// otherwise by coarse bucket ranges of 2^L2 sub-bins each (at most 256
// ranges; ranges grow when the table needs more).
// opts->log2_subbin and opts->split_bits, when nonzero, replace the two
// choices (already range-checked).  Sub-bins keep about 2^13 keys however
// many keys share a bucket (a table with long buckets then still sorts and
// probes every sub-bin in LDS), but no fewer than min_log2S buckets, and
// enough that 256 ranges of kMaxD2 sub-bins cover the table.
SplitParams split_params(uint32_t P, uint64_t n, uint64_t bound, const hg_build_opts* opts,
                         uint32_t min_log2S = 0) {
  SplitParams sp;
  const uint64_t buckets = bound > P ? bound - P : 1;
  uint32_t rho_log = 0;  // ceil(log2(keys per bucket)), at least 0
  while ((buckets << rho_log) < n) ++rho_log;
  const uint32_t lb = ceil_log2(bound < 2 ? 2 : bound);
  uint32_t l = hg::kLog2SMax > rho_log ? hg::kLog2SMax - rho_log : 0;
  if (l < min_log2S) l = min_log2S;
  if (lb > 18 && l < lb - 18) l = lb - 18;
  if (opts->log2_subbin != 0) l = opts->log2_subbin;
  sp.log2S = l;
  const uint64_t S = 1ull << l;
  const uint32_t l2 = opts->split_bits != 0 ? opts->split_bits : split_l2_bits();
  // A partition's last sub-bin may take up to 2^13 keys more than S buckets
  // hold on average.
  const uint64_t fits = ((1ull << l2) - 1) * S + std::max<uint64_t>(S, ((1ull << hg::kLog2SLds) / 2) >> rho_log);
  if (P > 1 && (buckets + P - 1) / P <= fits) {
    sp.mode = 0;
    sp.sh1 = 0;
    sp.nd1 = P;
    return sp;
  }
  uint32_t sh = l + l2;                // 2^l2 sub-bins per range
  if (lb > 8 && sh < lb - 8) sh = lb - 8;  // at most 256 ranges
  if (sh > l + 10) sh = l + 10;            // at most kMaxD2 sub-bins per range
  sp.mode = 1;
  sp.sh1 = sh;
  sp.nd1 = static_cast<uint32_t>((bound + (1ull << sh) - 1) >> sh);
  if (sp.nd1 == 0) sp.nd1 = 1;
  return sp;
}

uint32_t probe_log2W(hg_key_type kt, uint64_t n, uint64_t buckets) {
  const uint64_t kcap = hg::kProbeKeyCapBytes / key_bytes(kt);
  const double per_bucket = buckets ? static_cast<double>(n) / static_cast<double>(buckets) : 1.0;
  uint32_t l = hg::kMaxLog2W;
  while (l > 0 && static_cast<double>(1u << l) * (per_bucket * 1.1 + 0.01) > static_cast<double>(kcap)) --l;
  return l;
}

// The two splits of n keys (or queries) against layout (log2P, desc): the
// level-1 scatter into buf1 (level-1 counts already scanned and the plan
// written), then level-2 counts, scan and scatter into buf2.  perm1 / perm2
// (probes) receive each key's slot in its split tile at that level, which
// the tile gathers invert.
struct SplitBufs {
  uint32_t* counts1;
  uint32_t* bsums;
  hg::SegPlan* plan;
  uint32_t* counts2;
  void* buf1;
  void* buf2;
  uint32_t tiles1;
  uint32_t max_tiles2;
  uint32_t max_counts2;
  uint32_t max_subbins;
};

hg_status split_two_levels(const void* src, uint32_t n, hg_key_type kt, const SplitParams& sp, uint32_t log2P,
                           uint32_t P, const hg::PartDesc* desc, const SplitBufs& w, uint16_t* perm1,
                           uint16_t* perm2, const char* const names[4], hipStream_t s) {
  const int dig1 = sp.mode == 0 ? hg::DIG_PART : hg::DIG_COARSE;
  HG_LAUNCH(names[0], s,
            hg::launch_msplit(kt, 1, hg::OP_SCATTER, dig1, src, n, 0, nullptr, sp.nd1, log2P, P, desc, sp.sh1,
                              w.counts1, w.buf1, perm1, s));
  HG_LAUNCH(names[1], s,
            hg::launch_msplit(kt, 2, hg::OP_COUNT, hg::DIG_SUB, w.buf1, n, w.max_tiles2, w.plan, 0, log2P, P, desc,
                              sp.log2S, w.counts2, nullptr, nullptr, s));
  HG_LAUNCH(names[2], s, hg::launch_scan_exclusive(w.counts2, &w.plan->total_counts, w.max_counts2, w.bsums, s));
  HG_LAUNCH(names[3], s,
            hg::launch_msplit(kt, 2, hg::OP_SCATTER, hg::DIG_SUB, w.buf1, n, w.max_tiles2, w.plan, 0, log2P, P, desc,
                              sp.log2S, w.counts2, w.buf2, perm2, s));
  return HG_OK;
}

hg_status alloc_split(Allocs& mem, uint64_t n, hg_key_type kt, const SplitParams& sp, uint32_t P, uint64_t bound,
                      SplitBufs& w, uint64_t extra_scan) {
  const size_t ks = key_bytes(kt);
  const uint32_t tile2 = static_cast<uint32_t>(hg::l2_tile_keys(kt));
  w.tiles1 = hg::div_up(n, hg::kL1Tile);
  w.max_tiles2 = max_l2_tiles(n, tile2, sp.nd1);
  w.max_subbins = hg::div_up(bound, 1ull << sp.log2S) + sp.nd1;
  // A segment has at most kMaxD2 sub-bins; a coarse range of 2^sh1 buckets
  // (mode 1) at most 2^(sh1 - log2S).
  const uint64_t maxd2 = sp.mode == 1 ? std::min<uint64_t>(hg::kMaxD2, 1ull << (sp.sh1 - sp.log2S)) : hg::kMaxD2;
  w.max_counts2 = static_cast<uint32_t>(std::min<uint64_t>(maxd2 * w.max_tiles2, 0xFFFFFFFFull));
  const uint64_t len1 = static_cast<uint64_t>(std::max(sp.nd1, P)) * w.tiles1;
  const uint64_t scan_max = std::max<uint64_t>(std::max<uint64_t>(len1, w.max_counts2), extra_scan);
  void *c1 = nullptr, *bs = nullptr, *pl = nullptr, *c2 = nullptr, *b1 = nullptr, *b2 = nullptr;
  HG_TRY(mem.get(&c1, std::max<uint64_t>(len1, 1) * sizeof(uint32_t)), "allocate level-1 counts");
  HG_TRY(mem.get(&bs, (hg::div_up(scan_max, hg::kScanChunk) + 1) * sizeof(uint32_t)), "allocate scan workspace");
  HG_TRY(mem.get(&pl, hg::plan_bytes(sp.nd1, w.max_tiles2, w.max_subbins)), "allocate split plan");
  HG_TRY(mem.get(&c2, std::max<uint64_t>(w.max_counts2, 1) * sizeof(uint32_t)), "allocate level-2 counts");
  HG_TRY(mem.get(&b1, std::max<uint64_t>(n, 1) * ks), "allocate level-1 buffer");
  HG_TRY(mem.get(&b2, std::max<uint64_t>(n, 1) * ks), "allocate level-2 buffer");
  w.counts1 = static_cast<uint32_t*>(c1);
  w.bsums = static_cast<uint32_t*>(bs);
  w.plan = static_cast<hg::SegPlan*>(pl);
  w.counts2 = static_cast<uint32_t*>(c2);
  w.buf1 = b1;
  w.buf2 = b2;
  return HG_OK;
}

// Table layout from the scanned tile counts: the sizes from the ratio (or
// the plain V), or copied from another table's descriptors (`like`: the
// query table of hg_build_like).
hipError_t layout_of(const hg::PartDesc* like, const uint32_t* tile_base, uint32_t num_tiles, uint32_t P, uint32_t n,
                     const hg_build_opts* opts, uint64_t V_plain, uint32_t* po, uint32_t* bb, hg::PartDesc* desc,
                     hipStream_t s) {
  if (like != nullptr) return hg::launch_layout_like(tile_base, num_tiles, P, n, like, po, bb, desc, s);
  return hg::launch_layout(tile_base, num_tiles, P, n, opts->ratio_num, opts->ratio_den, V_plain, po, bb, desc, s);
}

// The LDS-sorted build (splits + one LDS counting sort per sub-bin).
hg_status build_sorted(const void* keys, uint32_t n, hg_key_type kt, uint32_t P, uint32_t log2P,
                       const hg_build_opts* opts, bool plain_V, uint64_t bound, const SplitParams& sp,
                       const hg::PartDesc* like, uint32_t* po, uint32_t* bb, hg::PartDesc* desc, uint32_t* offs,
                       void* keys_out, uint32_t* long_count, uint32_t* long_list, Allocs& mem, hipStream_t s) {
  SplitBufs w;
  hg_status st = alloc_split(mem, n, kt, sp, P, bound, w, 0);
  if (st != HG_OK) return st;
  const uint32_t tile2 = static_cast<uint32_t>(hg::l2_tile_keys(kt));
  const uint32_t max_subbins = w.max_subbins;
  if (sp.mode == 0) {
    HG_LAUNCH("split1_count", s,
              hg::launch_msplit(kt, 1, hg::OP_COUNT, hg::DIG_PART, keys, n, 0, nullptr, P, log2P, P, nullptr, 0,
                                w.counts1, nullptr, nullptr, s));
    HG_LAUNCH("split1_scan", s,
              hg::launch_scan_exclusive(w.counts1, nullptr, static_cast<uint64_t>(P) * w.tiles1, w.bsums, s));
    HG_LAUNCH("layout", s, layout_of(like, w.counts1, w.tiles1, P, n, opts, 0, po, bb, desc, s));
  } else {
    if (P > 1) {
      HG_LAUNCH("part_count", s, hg::launch_part_count(kt, keys, n, log2P, hg::div_up(n, hg::kTileKeys), w.counts1, s));
      HG_LAUNCH("part_scan", s,
                hg::launch_scan_exclusive(w.counts1, nullptr,
                                          static_cast<uint64_t>(P) * hg::div_up(n, hg::kTileKeys), w.bsums, s));
      HG_LAUNCH("layout", s, layout_of(like, w.counts1, hg::div_up(n, hg::kTileKeys), P, n, opts, 0, po, bb, desc, s));
    } else {
      HG_LAUNCH("layout", s,
                layout_of(like, nullptr, 0, 1, n, opts, plain_V ? opts->num_buckets : 0, po, bb, desc, s));
    }
    HG_LAUNCH("split1_count", s,
              hg::launch_msplit(kt, 1, hg::OP_COUNT, hg::DIG_COARSE, keys, n, 0, nullptr, sp.nd1, log2P, P, desc,
                                sp.sh1, w.counts1, nullptr, nullptr, s));
    HG_LAUNCH("split1_scan", s,
              hg::launch_scan_exclusive(w.counts1, nullptr, static_cast<uint64_t>(sp.nd1) * w.tiles1, w.bsums, s));
  }
  HG_LAUNCH("plan", s,
            hg::launch_plan(w.counts1, w.tiles1, sp.nd1, n, sp.mode, bb, bb + P, nullptr, sp.sh1, sp.log2S, tile2,
                            w.max_tiles2, w.max_subbins, offs, w.plan, s));
  static const char* const kNames[4] = {"split1_scatter", "split2_count", "split2_scan", "split2_scatter"};
  st = split_two_levels(keys, n, kt, sp, log2P, P, desc, w, nullptr, nullptr, kNames, s);
  if (st != HG_OK) return st;
  HeavyWork hw;
  st = alloc_heavy(mem, n, max_subbins, hw);
  if (st != HG_OK) return st;
  HG_LAUNCH("lds_build", s,
            hg::launch_lds_build(kt, w.buf2, w.plan, w.counts2, max_subbins, log2P, P, desc, offs, keys_out,
                                 long_count, long_list, hw.words, hw.max_chunks, hw.long_flags, s));
  return HG_OK;
}

// Sorted probe: the table's two splits on the queries, LDS-window counting,
// two gathers back to input order.
hg_status probe_sorted(const hg_table* t, const void* queries, uint32_t q, void* out, bool count, hipStream_t s) {
  const hg_key_type kt = t->kt;
  SplitParams sp;
  sp.mode = t->split_mode;
  sp.sh1 = t->sh1;
  sp.nd1 = t->nd1;
  sp.log2S = t->log2S;
  // The queries' sub-bins may be narrower than the table's: at most one LDS
  // window each (every query then hashes and is counted once), as long as a
  // coarse range keeps at most kMaxD2 of them.
  const uint32_t log2W = probe_log2W(kt, t->n, t->buckets_bound);
  if (sp.mode == 1) {
    while (sp.log2S > log2W && sp.sh1 - (sp.log2S - 1) <= 10) --sp.log2S;
    // Narrower sub-bins mean more level-2 digits per coarse range and
    // shorter runs in the level-2 split and gather; narrower ranges take
    // them back while the level-1 split keeps at most 256 digits (the
    // query split needs no ranges of the table's width: only its sub-bins
    // meet the table's windows).
    const uint64_t bound = t->buckets_bound;
    uint32_t sh = sp.sh1;
    while (sh > sp.log2S + split_l2_bits() && ((bound + (1ull << (sh - 1)) - 1) >> (sh - 1)) <= 256) --sh;
    if (sh != sp.sh1) {
      sp.sh1 = sh;
      sp.nd1 = static_cast<uint32_t>((t->buckets_bound + (1ull << sh) - 1) >> sh);
    }
  }
  Allocs mem(s);
  SplitBufs w;
  hg_status st = alloc_split(mem, q, kt, sp, t->P, t->buckets_bound, w, 0);
  if (st != HG_OK) return st;
  void *c2v = nullptr, *p1v = nullptr, *p2v = nullptr;
  HG_TRY(mem.get(&c2v, std::max<uint64_t>(q, 1) * sizeof(uint32_t)), "allocate split-order counts");
  HG_TRY(mem.get(&p1v, std::max<uint64_t>(q, 1) * sizeof(uint16_t)), "allocate level-1 permutation");
  HG_TRY(mem.get(&p2v, std::max<uint64_t>(q, 1) * sizeof(uint16_t)), "allocate level-2 permutation");
  const uint32_t tile2 = static_cast<uint32_t>(hg::l2_tile_keys(kt));
  const int dig1 = sp.mode == 0 ? hg::DIG_PART : hg::DIG_COARSE;
  const uint32_t max_subbins = w.max_subbins;
  HG_LAUNCH("qsplit1_count", s,
            hg::launch_msplit(kt, 1, hg::OP_COUNT, dig1, queries, q, 0, nullptr, sp.nd1, t->log2P, t->P, t->d_desc,
                              sp.sh1, w.counts1, nullptr, nullptr, s));
  HG_LAUNCH("qsplit1_scan", s,
            hg::launch_scan_exclusive(w.counts1, nullptr, static_cast<uint64_t>(sp.nd1) * w.tiles1, w.bsums, s));
  HG_LAUNCH("qplan", s,
            hg::launch_plan(w.counts1, w.tiles1, sp.nd1, q, sp.mode, t->d_bucket_base, t->d_bucket_base + t->P, nullptr,
                            sp.sh1, sp.log2S, tile2, w.max_tiles2, w.max_subbins, nullptr, w.plan, s));
  uint32_t* c2 = static_cast<uint32_t*>(c2v);
  uint16_t* perm1 = static_cast<uint16_t*>(p1v);
  uint16_t* perm2 = static_cast<uint16_t*>(p2v);
  static const char* const kNames[4] = {"qsplit1_scatter", "qsplit2_count", "qsplit2_scan", "qsplit2_scatter"};
  st = split_two_levels(queries, q, kt, sp, t->log2P, t->P, t->d_desc, w, perm1, perm2, kNames, s);
  if (st != HG_OK) return st;
  void* qv = nullptr;
  HG_TRY(mem.get(&qv, (3 + 2ull * (q / hg::probe_chunk_keys(kt) + 1)) * sizeof(uint32_t)), "allocate probe queue");
  HG_LAUNCH("lds_probe", s,
            hg::launch_lds_probe(kt, w.buf2, w.plan, w.counts2, max_subbins, q, t->log2P, t->P, t->d_desc,
                                 t->d_offsets, t->d_keys, t->d_unsorted, log2W, static_cast<uint32_t*>(qv), c2, s));
  // The level-1 buffer is dead once the level-2 split has read it: it takes
  // the counts in level-1 order (q words fit in q keys).  Counts travel as
  // bytes between these kernels when the table has no long bucket.
  uint32_t* c1 = static_cast<uint32_t*>(w.buf1);
  HG_LAUNCH("qgather2", s,
            hg::launch_tile_gather(kt, 2, perm2, c2, q, w.max_tiles2, w.plan, 0, w.counts2, t->d_unsorted, c1,
                                   hg::GATHER_STAGE, s));
  HG_LAUNCH("qgather1", s,
            hg::launch_tile_gather(kt, 1, perm1, c1, q, 0, nullptr, sp.nd1, w.counts1, t->d_unsorted, out,
                                   count ? hg::GATHER_COUNT : hg::GATHER_FOUND, s));
  return HG_OK;
}

bool use_sorted_probe(const hg_table* t, uint64_t q, uint32_t flags) {
  if (flags & HG_PROBE_DIRECT) return false;
  if (flags & HG_PROBE_SORTED) return true;
  // Large tables, or tables of long buckets (a direct probe searches each
  // query's bucket in global memory).
  return q >= (1ull << 20) && (t->buckets_bound >= (1ull << 22) || t->n >= 16 * t->buckets_bound);
}

hg_status probe(const hg_table* t, const void* d_queries, uint64_t q, void* d_out, bool count, uint32_t flags,
                hipStream_t s) {
  if (t == nullptr) return fail(HG_ERR_INVALID_ARG, "null table");
  if (t->batched) return fail(HG_ERR_INVALID_ARG, "a batched table is probed with hg_count_batched / hg_query_batched");
  if (q >= (1ull << 32)) return fail(HG_ERR_INVALID_ARG, "q = %llu is not below 2^32", (unsigned long long)q);
  if (q > 0 && (d_queries == nullptr || d_out == nullptr)) return fail(HG_ERR_INVALID_ARG, "null queries or output");
  if ((flags & ~(HG_PROBE_DIRECT | HG_PROBE_SORTED)) != 0 || flags == (HG_PROBE_DIRECT | HG_PROBE_SORTED))
    return fail(HG_ERR_INVALID_ARG, "unknown probe flags 0x%x", flags);
  if (q == 0) return HG_OK;
  if (use_sorted_probe(t, q, flags)) return probe_sorted(t, d_queries, static_cast<uint32_t>(q), d_out, count, s);
  HG_LAUNCH(count ? "probe_count" : "probe_found", s,
            hg::launch_probe(t->kt, count, t->d_keys, t->d_offsets, t->d_desc, t->log2P, t->P, t->d_unsorted,
                             d_queries, static_cast<uint32_t>(q), d_out, s));
  return HG_OK;
}

// Level-2 split, sub-bin builds and long-bucket sorting of keys already
// grouped into segments by `plan` (batched tables).
struct L2Bufs {
  hg::SegPlan* plan;
  uint32_t* counts2;
  uint32_t* bsums;
  void* buf2;
  uint32_t max_tiles2;
  uint32_t max_counts2;
  uint32_t max_subbins;
};

hg_status alloc_l2(Allocs& mem, uint64_t n, hg_key_type kt, uint32_t nseg, uint64_t bound, uint32_t log2S,
                   L2Bufs& w) {
  const uint32_t tile2 = static_cast<uint32_t>(hg::l2_tile_keys(kt));
  w.max_tiles2 = max_l2_tiles(n, tile2, nseg);
  w.max_subbins = hg::div_up(bound, 1ull << log2S) + nseg;
  w.max_counts2 = static_cast<uint32_t>(std::min<uint64_t>(static_cast<uint64_t>(hg::kMaxD2) * w.max_tiles2,
                                                           0xFFFFFFFFull));
  void *pl = nullptr, *c2 = nullptr, *bs = nullptr, *b2 = nullptr;
  HG_TRY(mem.get(&pl, hg::plan_bytes(nseg, w.max_tiles2, w.max_subbins)), "allocate split plan");
  HG_TRY(mem.get(&c2, std::max<uint64_t>(w.max_counts2, 1) * sizeof(uint32_t)), "allocate level-2 counts");
  HG_TRY(mem.get(&bs, (hg::div_up(w.max_counts2, hg::kScanChunk) + 1) * sizeof(uint32_t)), "allocate scan workspace");
  HG_TRY(mem.get(&b2, std::max<uint64_t>(n, 1) * key_bytes(kt)), "allocate level-2 buffer");
  w.plan = static_cast<hg::SegPlan*>(pl);
  w.counts2 = static_cast<uint32_t*>(c2);
  w.bsums = static_cast<uint32_t*>(bs);
  w.buf2 = b2;
  return HG_OK;
}

// Count, scan and scatter of the segments of w.plan (one descriptor per
// segment) from src into w.buf2; perm (probes) receives each key's slot in
// its split tile.
hg_status split_segments(const void* src, uint32_t n, hg_key_type kt, uint32_t log2S, const hg::PartDesc* desc,
                         const L2Bufs& w, uint16_t* perm, const char* const names[3], hipStream_t s) {
  HG_LAUNCH(names[0], s,
            hg::launch_msplit(kt, 2, hg::OP_COUNT, hg::DIG_SUB, src, n, w.max_tiles2, w.plan, 0, 0, 1, desc, log2S,
                              w.counts2, nullptr, nullptr, s));
  HG_LAUNCH(names[1], s, hg::launch_scan_exclusive(w.counts2, &w.plan->total_counts, w.max_counts2, w.bsums, s));
  HG_LAUNCH(names[2], s,
            hg::launch_msplit(kt, 2, hg::OP_SCATTER, hg::DIG_SUB, src, n, w.max_tiles2, w.plan, 0, 0, 1, desc, log2S,
                              w.counts2, w.buf2, perm, s));
  return HG_OK;
}

hg_status probe_batched(const hg_table* t, const void* d_queries, uint64_t q, const uint32_t* d_qo, void* d_out,
                        bool count, hipStream_t s) {
  if (t == nullptr) return fail(HG_ERR_INVALID_ARG, "null table");
  if (!t->batched) return fail(HG_ERR_INVALID_ARG, "not a batched table (probe it with hg_count / hg_query)");
  if (q >= (1ull << 32)) return fail(HG_ERR_INVALID_ARG, "q = %llu is not below 2^32", (unsigned long long)q);
  if (d_qo == nullptr) return fail(HG_ERR_INVALID_ARG, "null query offsets");
  if (q > 0 && (d_queries == nullptr || d_out == nullptr)) return fail(HG_ERR_INVALID_ARG, "null queries or output");
  if (q == 0) return HG_OK;
  const hg_key_type kt = t->kt;
  const uint32_t T = t->P, q32 = static_cast<uint32_t>(q);
  Allocs mem(s);
  L2Bufs w;
  hg_status st = alloc_l2(mem, q, kt, T, t->buckets_bound, t->log2S, w);
  if (st != HG_OK) return st;
  void *qov = nullptr, *pv = nullptr, *c2v = nullptr;
  HG_TRY(mem.get(&qov, (static_cast<uint64_t>(T) + 1) * sizeof(uint32_t)), "allocate query offsets");
  HG_TRY(mem.get(&pv, q * sizeof(uint16_t)), "allocate permutation");
  HG_TRY(mem.get(&c2v, q * sizeof(uint32_t)), "allocate split-order counts");
  uint32_t* qo = static_cast<uint32_t*>(qov);
  uint16_t* perm = static_cast<uint16_t*>(pv);
  uint32_t* c2 = static_cast<uint32_t*>(c2v);
  const uint32_t tile2 = static_cast<uint32_t>(hg::l2_tile_keys(kt));
  HG_LAUNCH("bq_offsets", s, hg::launch_batch_layout(d_qo, T, q32, 1, 1, qo, nullptr, nullptr, s));
  HG_LAUNCH("bq_plan", s,
            hg::launch_plan(nullptr, 0, T, q32, 2, t->d_bucket_base, t->d_bucket_base + T, qo, 0, t->log2S, tile2,
                            w.max_tiles2, w.max_subbins, nullptr, w.plan, s));
  static const char* const kNames[3] = {"bqsplit_count", "bqsplit_scan", "bqsplit_scatter"};
  st = split_segments(d_queries, q32, kt, t->log2S, t->d_desc, w, perm, kNames, s);
  if (st != HG_OK) return st;
  const uint32_t max_subbins = w.max_subbins;
  void* qv = nullptr;
  HG_TRY(mem.get(&qv, (3 + 2ull * (q / hg::probe_chunk_keys(kt) + 1)) * sizeof(uint32_t)), "allocate probe queue");
  HG_LAUNCH("blds_probe", s,
            hg::launch_lds_probe(kt, w.buf2, w.plan, w.counts2, max_subbins, q32, 0, 1, t->d_desc, t->d_offsets,
                                 t->d_keys, t->d_unsorted, probe_log2W(kt, t->n, t->buckets_bound),
                                 static_cast<uint32_t*>(qv), c2, s));
  HG_LAUNCH("bqgather", s,
            hg::launch_tile_gather(kt, 2, perm, c2, q32, w.max_tiles2, w.plan, 0, w.counts2, t->d_unsorted, d_out,
                                   count ? hg::GATHER_COUNT : hg::GATHER_FOUND, s));
  return HG_OK;
}

hg_status check_tuning(const hg_build_opts* opts) {
  if (opts->log2_subbin != 0 && (opts->log2_subbin < hg::kLog2SMin || opts->log2_subbin > hg::kLog2SMax))
    return fail(HG_ERR_INVALID_ARG, "log2_subbin = %u outside [%u, %u]", opts->log2_subbin, hg::kLog2SMin,
                hg::kLog2SMax);
  if (opts->split_bits != 0 && (opts->split_bits < 7 || opts->split_bits > 10))
    return fail(HG_ERR_INVALID_ARG, "split_bits = %u outside [7, 10]", opts->split_bits);
  return HG_OK;
}

}  // namespace

extern "C" {

// The build of hg_build, or of hg_build_like when `like` is given (then the
// layout, hence every key's bucket, is the one of `like`).
static hg_status build_impl(const void* d_keys, uint64_t n, hg_key_type kt, const hg_build_opts* opts,
                            const hg_table* like, hipStream_t stream, hg_table** out) {
  if (out == nullptr || opts == nullptr) return fail(HG_ERR_INVALID_ARG, "null opts or out");
  if (check_tuning(opts) != HG_OK) return HG_ERR_INVALID_ARG;
  hg_status st = check_n_P(n, kt, opts->P);
  if (st != HG_OK) return st;
  if (n > 0 && d_keys == nullptr) return fail(HG_ERR_INVALID_ARG, "null keys");
  if ((opts->flags & ~(HG_BUILD_ATOMIC | HG_BUILD_SORTED)) != 0 ||
      opts->flags == (HG_BUILD_ATOMIC | HG_BUILD_SORTED))
    return fail(HG_ERR_INVALID_ARG, "unknown build flags 0x%x", opts->flags);
  const uint32_t P = opts->P;
  const bool plain_V = (P == 1 && opts->num_buckets != 0);
  uint64_t bound;
  if (plain_V) {
    if (opts->num_buckets > 0xFFFFFFFEull) return fail(HG_ERR_INVALID_ARG, "num_buckets exceeds 2^32 - 2");
    bound = opts->num_buckets;
  } else {
    if (opts->ratio_num == 0 || opts->ratio_den == 0) return fail(HG_ERR_INVALID_ARG, "zero table ratio");
    // sum_p max(1, floor(n_p * num / den)) <= floor(n * num / den) + P.
    bound = n * static_cast<uint64_t>(opts->ratio_num) / opts->ratio_den + P;
    if (bound > 0xFFFFFFFEull) return fail(HG_ERR_INVALID_ARG, "table ratio gives more than 2^32 - 2 buckets");
  }
  if (like != nullptr) bound = like->buckets_bound;  // the same buckets
  const hg::PartDesc* like_desc = like != nullptr ? like->d_desc : nullptr;

  const uint32_t n32 = static_cast<uint32_t>(n);
  const uint32_t log2P = log2_of(P);
  const size_t ks = key_bytes(kt);
  const uint32_t num_tiles = hg::div_up(n, hg::kTileKeys);
  int device = 0;
  HG_TRY(current_device(&device), "hipGetDevice");

  Allocs mem(stream);
  void *keys_out = nullptr, *offsets = nullptr, *meta = nullptr;
  const size_t meta_bytes =
      2 * sizeof(uint32_t) * (P + 1) + 8 + sizeof(hg::PartDesc) * P + sizeof(uint32_t) * hg::kUnsortedWords;
  HG_TRY(mem.get(&keys_out, n * ks), "allocate table keys");
  HG_TRY(mem.get(&offsets, (bound + 1) * sizeof(uint32_t)), "allocate table offsets");
  HG_TRY(mem.get(&meta, meta_bytes), "allocate table metadata");
  uint32_t* po = static_cast<uint32_t*>(meta);
  uint32_t* bb = po + (P + 1);
  uintptr_t dp = reinterpret_cast<uintptr_t>(bb + (P + 1));
  dp = (dp + 7) & ~static_cast<uintptr_t>(7);
  hg::PartDesc* desc = reinterpret_cast<hg::PartDesc*>(dp);
  uint32_t* unsorted = reinterpret_cast<uint32_t*>(desc + P);

  // Long-bucket bookkeeping: at most n / (kLongT + 1) buckets exceed kLongT.
  void* longv = nullptr;
  const uint64_t long_cap = hg::long_list_cap(n);
  HG_TRY(mem.get(&longv, (hg::kLongCtr + long_cap) * sizeof(uint32_t)), "allocate long-bucket list");
  uint32_t* long_ctr = static_cast<uint32_t*>(longv);
  uint32_t* long_list = long_ctr + hg::kLongCtr;
  HG_LAUNCH("zero_long", stream, hg::launch_fill_u32(long_ctr, hg::kLongCtr, 0u, stream));
  HG_LAUNCH("zero_long", stream, hg::launch_fill_u32(long_ctr + 4, 1, static_cast<uint32_t>(long_cap), stream));
  HG_LAUNCH("zero_unsorted", stream, hg::launch_fill_u32(unsorted, 1, 0u, stream));

  const SplitParams sp = split_params(P, n, bound, opts);
  uint32_t* offs = static_cast<uint32_t*>(offsets);
  // Large tables, or tables of long buckets (the atomic histogram and
  // scatter then serialise on few counters).
  const bool sorted = (opts->flags & HG_BUILD_SORTED) != 0 ||
                      ((opts->flags & HG_BUILD_ATOMIC) == 0 && n >= (1ull << 20) &&
                       (bound >= (1ull << 22) || n >= 16 * bound));
  if (sorted) {
    st = build_sorted(d_keys, n32, kt, P, log2P, opts, plain_V, bound, sp, like_desc, po, bb, desc, offs, keys_out,
                      long_ctr, long_list, mem, stream);
    if (st != HG_OK) return st;
  } else {
  const uint64_t part_elems = P > 1 ? static_cast<uint64_t>(P) * num_tiles : 0;
  const uint64_t scan_max = part_elems > bound ? part_elems : bound;
  void *tile_counts = nullptr, *buffer = nullptr, *bsums = nullptr;
  HG_TRY(mem.get(&bsums, (hg::div_up(scan_max, hg::kScanChunk) + 1) * sizeof(uint32_t)), "allocate scan workspace");

  const void* src = d_keys;
  if (P > 1) {
    HG_TRY(mem.get(&tile_counts, part_elems * sizeof(uint32_t)), "allocate tile counts");
    HG_TRY(mem.get(&buffer, n * ks), "allocate partition buffer");
    st = run_partition(d_keys, n32, kt, log2P, num_tiles, static_cast<uint32_t*>(tile_counts),
                       static_cast<uint32_t*>(bsums), buffer, stream);
    if (st != HG_OK) return st;
    HG_LAUNCH("layout", stream,
              layout_of(like_desc, static_cast<uint32_t*>(tile_counts), num_tiles, P, n32, opts, 0, po, bb, desc,
                        stream));
    src = buffer;
  } else {
    HG_LAUNCH("layout", stream,
              layout_of(like_desc, nullptr, 0, 1, n32, opts, plain_V ? opts->num_buckets : 0, po, bb, desc, stream));
  }

  HG_LAUNCH("zero_counts", stream, hg::launch_fill_u32(offs, bound + 1, 0u, stream));
  HG_LAUNCH("bucket_hist", stream, hg::launch_hist(kt, src, n32, log2P, P, desc, offs + 1, stream));
  HG_LAUNCH("bucket_scan", stream,
            hg::launch_scan_exclusive(offs + 1, bb + P, bound, static_cast<uint32_t*>(bsums), stream));
  HG_LAUNCH("bucket_scatter", stream, hg::launch_scatter(kt, src, n32, log2P, P, desc, offs + 1, keys_out, stream));
  HG_LAUNCH("find_long", stream, hg::launch_find_long(offs, bb + P, bound, long_ctr, long_list, stream));
  }
  void* bigv = nullptr;
  HG_TRY(mem.get(&bigv, hg::big_words(n, static_cast<uint32_t>(ks)) * sizeof(uint32_t)),
         "allocate long-bucket chunk lists");
  HG_LAUNCH("long_sort", stream,
            hg::launch_long_sort(kt, offs, long_ctr, long_list, keys_out, unsorted, static_cast<uint32_t*>(bigv), n,
                                 stream));

  hg_table* t = new hg_table();
  t->device = device;
  t->stream = stream;
  t->kt = kt;
  t->n = n;
  t->P = P;
  t->log2P = log2P;
  t->buckets_bound = bound;
  t->d_keys = keys_out;
  t->d_offsets = offs;
  t->d_meta = meta;
  t->d_part_offsets = po;
  t->d_bucket_base = bb;
  t->d_desc = desc;
  t->d_unsorted = unsorted;
  t->split_mode = sp.mode;
  t->sh1 = sp.sh1;
  t->nd1 = sp.nd1;
  t->log2S = sp.log2S;
  t->batched = false;
  t->id = g_next_table_id.fetch_add(1);
  t->like_id = like != nullptr ? like->id : 0;
  t->have_num_buckets = false;
  t->num_buckets = 0;
  t->has_long = 0;
  t->blocks = {mem.release(keys_out), mem.release(offsets), mem.release(meta)};
  *out = t;
  return HG_OK;
}

hg_status hg_build(const void* d_keys, uint64_t n, hg_key_type kt, const hg_build_opts* opts, hipStream_t stream,
                   hg_table** out) {
  return build_impl(d_keys, n, kt, opts, nullptr, stream, out);
}

hg_status hg_build_like(const hg_table* table, const void* d_keys, uint64_t n, hipStream_t stream, hg_table** out) {
  if (table == nullptr) return fail(HG_ERR_INVALID_ARG, "null table");
  if (table->batched) return fail(HG_ERR_INVALID_ARG, "a batched table has no single layout to copy");
  hg_build_opts o = {};
  o.P = table->P;
  o.ratio_num = 1;
  o.ratio_den = 1;
  return build_impl(d_keys, n, table->kt, &o, table, stream, out);
}

hg_status hg_intersect(const hg_table* table, const hg_table* queries, uint32_t* d_counts, hipStream_t stream) {
  if (table == nullptr || queries == nullptr) return fail(HG_ERR_INVALID_ARG, "null table");
  if (queries->like_id != table->id)
    return fail(HG_ERR_INVALID_ARG, "the query table was not built like this table (hg_build_like)");
  if (queries->n == 0) return HG_OK;
  if (d_counts == nullptr) return fail(HG_ERR_INVALID_ARG, "null counts");
  // Bucket g of both tables holds the keys that hash to g, and the query
  // table lists its keys bucket by bucket: each query key is counted in the
  // table's list of the same bucket, the lists of consecutive buckets in
  // turn.
  HG_LAUNCH("intersect", stream,
            hg::launch_probe(table->kt, true, table->d_keys, table->d_offsets, table->d_desc, table->log2P, table->P,
                             table->d_unsorted, queries->d_keys, static_cast<uint32_t>(queries->n), d_counts,
                             stream));
  return HG_OK;
}

hg_status hg_count(const hg_table* table, const void* d_queries, uint64_t q, uint32_t* d_counts, hipStream_t stream) {
  return probe(table, d_queries, q, d_counts, true, 0, stream);
}

hg_status hg_query(const hg_table* table, const void* d_queries, uint64_t q, uint8_t* d_found, hipStream_t stream) {
  return probe(table, d_queries, q, d_found, false, 0, stream);
}

hg_status hg_count_ex(const hg_table* table, const void* d_queries, uint64_t q, uint32_t* d_counts, uint32_t flags,
                      hipStream_t stream) {
  return probe(table, d_queries, q, d_counts, true, flags, stream);
}

hg_status hg_query_ex(const hg_table* table, const void* d_queries, uint64_t q, uint8_t* d_found, uint32_t flags,
                      hipStream_t stream) {
  return probe(table, d_queries, q, d_found, false, flags, stream);
}

hg_status hg_build_batched(const void* d_keys, uint64_t n, hg_key_type kt, uint32_t num_tables,
                           const uint32_t* d_table_offsets, const hg_build_opts* opts, hipStream_t stream,
                           hg_table** out) {
  if (out == nullptr || opts == nullptr) return fail(HG_ERR_INVALID_ARG, "null opts or out");
  if (check_tuning(opts) != HG_OK) return HG_ERR_INVALID_ARG;
  hg_status st = check_n_P(n, kt, 1);
  if (st != HG_OK) return st;
  const uint32_t T = num_tables;
  if (T == 0 || T > hg::kMaxTables) return fail(HG_ERR_INVALID_ARG, "num_tables = %u outside [1, 2^22]", T);
  if (d_table_offsets == nullptr) return fail(HG_ERR_INVALID_ARG, "null table offsets");
  if (n > 0 && d_keys == nullptr) return fail(HG_ERR_INVALID_ARG, "null keys");
  if (opts->P != 1) return fail(HG_ERR_INVALID_ARG, "batched tables take P = 1 (got %u)", opts->P);
  if (opts->num_buckets != 0) return fail(HG_ERR_INVALID_ARG, "batched tables take their size from the ratio");
  if ((opts->flags & ~(HG_BUILD_ATOMIC | HG_BUILD_SORTED)) != 0)
    return fail(HG_ERR_INVALID_ARG, "unknown build flags 0x%x", opts->flags);
  if (opts->flags & HG_BUILD_ATOMIC) return fail(HG_ERR_UNSUPPORTED, "batched tables use the sorted build");
  if (opts->ratio_num == 0 || opts->ratio_den == 0) return fail(HG_ERR_INVALID_ARG, "zero table ratio");
  // sum_t max(1, floor(n_t * num / den)) <= floor(n * num / den) + T.
  const uint64_t bound = n * static_cast<uint64_t>(opts->ratio_num) / opts->ratio_den + T;
  if (bound > 0xFFFFFFFEull) return fail(HG_ERR_INVALID_ARG, "table ratio gives more than 2^32 - 2 buckets");

  const uint32_t n32 = static_cast<uint32_t>(n);
  const size_t ks = key_bytes(kt);
  int device = 0;
  HG_TRY(current_device(&device), "hipGetDevice");
  Allocs mem(stream);
  void *keys_out = nullptr, *offsets = nullptr, *meta = nullptr, *longv = nullptr;
  const size_t meta_bytes =
      2 * sizeof(uint32_t) * (static_cast<size_t>(T) + 1) + 8 + sizeof(hg::PartDesc) * T +
      sizeof(uint32_t) * hg::kUnsortedWords;
  HG_TRY(mem.get(&keys_out, std::max<uint64_t>(n, 1) * ks), "allocate table keys");
  HG_TRY(mem.get(&offsets, (bound + 1) * sizeof(uint32_t)), "allocate table offsets");
  HG_TRY(mem.get(&meta, meta_bytes), "allocate table metadata");
  uint32_t* po = static_cast<uint32_t*>(meta);
  uint32_t* bb = po + (T + 1);
  uintptr_t dp = reinterpret_cast<uintptr_t>(bb + (T + 1));
  dp = (dp + 7) & ~static_cast<uintptr_t>(7);
  hg::PartDesc* desc = reinterpret_cast<hg::PartDesc*>(dp);
  uint32_t* unsorted = reinterpret_cast<uint32_t*>(desc + T);
  const uint64_t long_cap = hg::long_list_cap(n);
  HG_TRY(mem.get(&longv, (hg::kLongCtr + long_cap) * sizeof(uint32_t)), "allocate long-bucket list");
  uint32_t* long_ctr = static_cast<uint32_t*>(longv);
  uint32_t* long_list = long_ctr + hg::kLongCtr;
  uint32_t* offs = static_cast<uint32_t*>(offsets);
  HG_LAUNCH("zero_long", stream, hg::launch_fill_u32(long_ctr, hg::kLongCtr, 0u, stream));
  HG_LAUNCH("zero_long", stream, hg::launch_fill_u32(long_ctr + 4, 1, static_cast<uint32_t>(long_cap), stream));
  HG_LAUNCH("zero_unsorted", stream, hg::launch_fill_u32(unsorted, 1, 0u, stream));
  HG_LAUNCH("batch_layout", stream,
            hg::launch_batch_layout(d_table_offsets, T, n32, opts->ratio_num, opts->ratio_den, po, bb, desc, stream));

  // Sub-bin size from the batch's keys per bucket; a table's sub-bins stay at
  // 2^kLog2SMin buckets or more, so that its segment has at most kMaxD2.
  const SplitParams sp = split_params(1, n, bound, opts, hg::kLog2SMin);
  L2Bufs w;
  st = alloc_l2(mem, n, kt, T, bound, sp.log2S, w);
  if (st != HG_OK) return st;
  const uint32_t tile2 = static_cast<uint32_t>(hg::l2_tile_keys(kt));
  HG_LAUNCH("bplan", stream,
            hg::launch_plan(nullptr, 0, T, n32, 2, bb, bb + T, po, 0, sp.log2S, tile2, w.max_tiles2, w.max_subbins,
                            offs, w.plan, stream));
  static const char* const kNames[3] = {"bsplit_count", "bsplit_scan", "bsplit_scatter"};
  st = split_segments(d_keys, n32, kt, sp.log2S, desc, w, nullptr, kNames, stream);
  if (st != HG_OK) return st;
  const uint32_t max_subbins = w.max_subbins;
  HeavyWork hw;
  st = alloc_heavy(mem, n, max_subbins, hw);
  if (st != HG_OK) return st;
  HG_LAUNCH("blds_build", stream,
            hg::launch_lds_build(kt, w.buf2, w.plan, w.counts2, max_subbins, 0, 1, desc, offs, keys_out, long_ctr,
                                 long_list, hw.words, hw.max_chunks, hw.long_flags, stream));
  void* bigv = nullptr;
  HG_TRY(mem.get(&bigv, hg::big_words(n, static_cast<uint32_t>(ks)) * sizeof(uint32_t)),
         "allocate long-bucket chunk lists");
  HG_LAUNCH("long_sort", stream,
            hg::launch_long_sort(kt, offs, long_ctr, long_list, keys_out, unsorted, static_cast<uint32_t*>(bigv), n,
                                 stream));

  hg_table* t = new hg_table();
  t->device = device;
  t->stream = stream;
  t->kt = kt;
  t->n = n;
  t->P = T;
  t->log2P = 0;
  t->buckets_bound = bound;
  t->d_keys = keys_out;
  t->d_offsets = offs;
  t->d_meta = meta;
  t->d_part_offsets = po;
  t->d_bucket_base = bb;
  t->d_desc = desc;
  t->d_unsorted = unsorted;
  t->split_mode = 2;
  t->sh1 = 0;
  t->nd1 = T;
  t->log2S = sp.log2S;
  t->batched = true;
  t->id = g_next_table_id.fetch_add(1);
  t->like_id = 0;
  t->have_num_buckets = false;
  t->num_buckets = 0;
  t->has_long = 0;
  t->blocks = {mem.release(keys_out), mem.release(offsets), mem.release(meta)};
  *out = t;
  return HG_OK;
}

hg_status hg_count_batched(const hg_table* table, const void* d_queries, uint64_t q, const uint32_t* d_query_offsets,
                           uint32_t* d_counts, hipStream_t stream) {
  return probe_batched(table, d_queries, q, d_query_offsets, d_counts, true, stream);
}

hg_status hg_query_batched(const hg_table* table, const void* d_queries, uint64_t q, const uint32_t* d_query_offsets,
                           uint8_t* d_found, hipStream_t stream) {
  return probe_batched(table, d_queries, q, d_query_offsets, d_found, false, stream);
}

hg_status hg_bin_partition(const void* d_keys, uint64_t n, hg_key_type kt, uint32_t P, void* d_out_keys,
                           uint32_t* d_part_offsets, hipStream_t stream) {
  hg_status st = check_n_P(n, kt, P);
  if (st != HG_OK) return st;
  if (d_part_offsets == nullptr) return fail(HG_ERR_INVALID_ARG, "null part_offsets");
  if (n > 0 && (d_keys == nullptr || d_out_keys == nullptr)) return fail(HG_ERR_INVALID_ARG, "null keys");
  const uint32_t n32 = static_cast<uint32_t>(n);
  const uint32_t log2P = log2_of(P);
  const uint32_t num_tiles = hg::div_up(n, hg::kTileKeys);
  const uint64_t elems = static_cast<uint64_t>(P) * num_tiles;
  Allocs mem(stream);
  void *tile_counts = nullptr, *bsums = nullptr;
  HG_TRY(mem.get(&tile_counts, elems * sizeof(uint32_t)), "allocate tile counts");
  HG_TRY(mem.get(&bsums, (hg::div_up(elems, hg::kScanChunk) + 1) * sizeof(uint32_t)), "allocate scan workspace");
  st = run_partition(d_keys, n32, kt, log2P, num_tiles, static_cast<uint32_t*>(tile_counts),
                     static_cast<uint32_t*>(bsums), d_out_keys, stream);
  if (st != HG_OK) return st;
  HG_LAUNCH("part_offsets", stream,
            hg::launch_layout(static_cast<uint32_t*>(tile_counts), num_tiles, P, n32, 1, 1, 0, d_part_offsets,
                              nullptr, nullptr, stream));
  return HG_OK;
}

}  // extern "C"

namespace {

// Device scratch of hg_bin_partition_noalloc: the per-tile partition counts,
// then the scan's block sums.  Every device the library runs on holds its own
// copy until the process ends.  In host code `scratch` is only a stand-in for
// the symbol; the device address comes from hipGetSymbolAddress, once per
// device (scratch_on).
constexpr uint64_t kScratchWords = (uint64_t(1) << 20) + 1024;  // 4 MiB + 4 KiB
static __device__ __align__(256) uint32_t scratch[kScratchWords];

std::mutex g_scratch_mu;
std::map<int, uint32_t*> g_scratch_ptr;

// The address of device `dev`'s scratch (that device must be current).
hipError_t scratch_on(int dev, uint32_t** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
  *out = static_cast<uint32_t*>(p);
  return hipSuccess;
}

// hg_bin_partition_noalloc takes at most kScratchCounts tile counts; padded
// to 256 bytes and followed by the scan's block sums they fit the scratch.
constexpr uint64_t kScratchCounts = uint64_t(1) << 20;
static_assert(kScratchCounts + kScratchCounts / hg::kScanChunk + 1 <= kScratchWords, "scratch holds counts and sums");

}  // namespace

extern "C" {

hg_status hg_bin_partition_noalloc(const void* d_keys, uint64_t n, hg_key_type kt, uint32_t P, void* d_out_keys,
                                   uint32_t* d_part_offsets, hipStream_t stream) {
  hg_status st = check_n_P(n, kt, P);
  if (st != HG_OK) return st;
  if (d_part_offsets == nullptr) return fail(HG_ERR_INVALID_ARG, "null part_offsets");
  if (n > 0 && (d_keys == nullptr || d_out_keys == nullptr)) return fail(HG_ERR_INVALID_ARG, "null keys");
  const uint64_t need = static_cast<uint64_t>(P) * hg::div_up(n, hg::kTileKeys);
  if (need > kScratchCounts)
    return fail(HG_ERR_INVALID_ARG,
                "hg_bin_partition_noalloc: n = %llu keys in P = %u partitions need %llu tile counts of scratch "
                "(P * ceil(n / %d)), more than its %llu; use hg_bin_partition",
                (unsigned long long)n, P, (unsigned long long)need, hg::kTileKeys,
                (unsigned long long)kScratchCounts);
  int dev = 0;
  HG_TRY(hipGetDevice(&dev), "hipGetDevice");
  uint32_t* ws = nullptr;
  HG_TRY(scratch_on(dev, &ws), "hipGetSymbolAddress(scratch)");
  const uint32_t n32 = static_cast<uint32_t>(n);
  const uint32_t num_tiles = hg::div_up(n, hg::kTileKeys);
  const uint64_t elems = static_cast<uint64_t>(P) * num_tiles;
  // The count pass writes every (partition, tile) entry and the scan every
  // block sum, so nothing left by an earlier call is read.
  uint32_t* tile_counts = ws;
  uint32_t* bsums = ws + (elems + 63) / 64 * 64;
  st = run_partition(d_keys, n32, kt, log2_of(P), num_tiles, tile_counts, bsums, d_out_keys, stream);
  if (st != HG_OK) return st;
  HG_LAUNCH("part_offsets", stream,
            hg::launch_layout(tile_counts, num_tiles, P, n32, 1, 1, 0, d_part_offsets, nullptr, nullptr, stream));
  return HG_OK;
}

hg_status hg_bin_partition_balanced(const void* d_keys, uint64_t n, hg_key_type kt, uint32_t P, uint64_t hash_range,
                                    uint32_t num_bins, void* d_out_keys, uint32_t* d_part_offsets,
                                    uint32_t* d_bin_splits, hipStream_t stream) {
  if (kt != HG_KEY_U32 && kt != HG_KEY_U64) return fail(HG_ERR_INVALID_ARG, "unknown key type %d", (int)kt);
  if (n >= (1ull << 32)) return fail(HG_ERR_INVALID_ARG, "n = %llu is not below 2^32", (unsigned long long)n);
  if (P == 0 || P > hg::kMaxP) return fail(HG_ERR_INVALID_ARG, "P = %u outside [1, %u]", P, hg::kMaxP);
  if (hash_range == 0 || hash_range >= (1ull << 32))
    return fail(HG_ERR_INVALID_ARG, "hash range %llu outside [1, 2^32)", (unsigned long long)hash_range);
  if (num_bins > hg::kMaxBins) return fail(HG_ERR_INVALID_ARG, "num_bins = %u exceeds %u", num_bins, hg::kMaxBins);
  if (d_part_offsets == nullptr || d_bin_splits == nullptr) return fail(HG_ERR_INVALID_ARG, "null outputs");
  if (n > 0 && (d_keys == nullptr || d_out_keys == nullptr)) return fail(HG_ERR_INVALID_ARG, "null keys");
  uint64_t bins = num_bins;
  if (bins == 0) {  // ceil(sqrt(HR)), at most kMaxBins
    bins = 1;
    while (bins * bins < hash_range && bins < hg::kMaxBins) ++bins;
  }
  const uint32_t HR = static_cast<uint32_t>(hash_range);
  const uint32_t bin_size = static_cast<uint32_t>((hash_range + bins - 1) / bins);
  const uint32_t nbins = static_cast<uint32_t>((hash_range + bin_size - 1) / bin_size);
  const uint32_t n32 = static_cast<uint32_t>(n);
  const uint32_t tiles = hg::div_up(n, hg::kL1Tile);
  const uint64_t tile_elems = static_cast<uint64_t>(P) * tiles;
  Allocs mem(stream);
  void *bc = nullptr, *bs = nullptr, *tc = nullptr, *rd = nullptr;
  HG_TRY(mem.get(&bc, (static_cast<uint64_t>(nbins) + 1) * sizeof(uint32_t)), "allocate bin counts");
  HG_TRY(mem.get(&bs, (hg::div_up(std::max<uint64_t>(nbins, tile_elems), hg::kScanChunk) + 1) * sizeof(uint32_t)),
         "allocate scan workspace");
  HG_TRY(mem.get(&tc, std::max<uint64_t>(tile_elems, 1) * sizeof(uint32_t)), "allocate tile counts");
  HG_TRY(mem.get(&rd, sizeof(hg::PartDesc) + (hg::kMaxP + 1) * sizeof(uint32_t)), "allocate range descriptor");
  uint32_t* bin_counts = static_cast<uint32_t*>(bc);
  uint32_t* bsums = static_cast<uint32_t*>(bs);
  uint32_t* tile_counts = static_cast<uint32_t*>(tc);
  hg::PartDesc* rdesc = static_cast<hg::PartDesc*>(rd);
  HG_LAUNCH("bin_zero", stream, hg::launch_fill_u32(bin_counts, nbins, 0u, stream));
  HG_LAUNCH("bin_hist", stream, hg::launch_bin_hist(kt, d_keys, n32, HR, bin_size, nbins, bin_counts, stream));
  HG_LAUNCH("bin_scan", stream, hg::launch_scan_exclusive(bin_counts, nullptr, nbins, bsums, stream));
  HG_LAUNCH("bin_splits", stream,
            hg::launch_range_splits(bin_counts, nbins, n32, P, HR, bin_size, d_bin_splits, rdesc, stream));
  HG_LAUNCH("range_count", stream,
            hg::launch_msplit(kt, 1, hg::OP_COUNT, hg::DIG_RANGE, d_keys, n32, 0, nullptr, P, 0, 1, rdesc, 0,
                              tile_counts, nullptr, nullptr, stream));
  HG_LAUNCH("range_scan", stream, hg::launch_scan_exclusive(tile_counts, nullptr, tile_elems, bsums, stream));
  HG_LAUNCH("range_offsets", stream,
            hg::launch_layout(tile_counts, tiles, P, n32, 1, 1, 0, d_part_offsets, nullptr, nullptr, stream));
  HG_LAUNCH("range_scatter", stream,
            hg::launch_msplit(kt, 1, hg::OP_SCATTER, hg::DIG_RANGE, d_keys, n32, 0, nullptr, P, 0, 1, rdesc, 0,
                              tile_counts, d_out_keys, nullptr, stream));
  return HG_OK;
}

hg_status hg_hash_bucket(const void* d_keys, uint64_t n, hg_key_type kt, uint64_t V, uint64_t* d_hash,
                         uint32_t* d_bucket, hipStream_t stream) {
  hg_status st = check_n_P(n, kt, 1);
  if (st != HG_OK) return st;
  if (V == 0 || V > 0xFFFFFFFFull) return fail(HG_ERR_INVALID_ARG, "V = %llu outside [1, 2^32)", (unsigned long long)V);
  if (n > 0 && d_keys == nullptr) return fail(HG_ERR_INVALID_ARG, "null keys");
  if (n == 0 || (d_hash == nullptr && d_bucket == nullptr)) return HG_OK;
  HG_LAUNCH("hash_bucket", stream,
            hg::launch_hash_bucket(kt, d_keys, static_cast<uint32_t>(n), static_cast<uint32_t>(V), d_hash, d_bucket,
                                   stream));
  return HG_OK;
}

hg_status hg_table_info(const hg_table* table, hg_table_desc* desc) {
  if (table == nullptr || desc == nullptr) return fail(HG_ERR_INVALID_ARG, "null table or desc");
  hg_table* t = const_cast<hg_table*>(table);
  {
    std::lock_guard<std::mutex> lk(t->mu);
    if (!t->have_num_buckets) {
      uint32_t nb = 0, hl = 0;
      HG_TRY(hipMemcpyAsync(&nb, t->d_bucket_base + t->P, sizeof(nb), hipMemcpyDeviceToHost, t->stream),
             "read bucket count");
      HG_TRY(hipMemcpyAsync(&hl, t->d_unsorted + hg::kHasLongWord, sizeof(hl), hipMemcpyDeviceToHost, t->stream),
             "read long-bucket word");
      HG_TRY(hipStreamSynchronize(t->stream), "wait for build");
      t->num_buckets = nb;
      t->has_long = hl;
      t->have_num_buckets = true;
    }
  }
  desc->n = t->n;
  desc->num_buckets = t->num_buckets;
  desc->P = t->P;
  desc->key_type = static_cast<uint32_t>(t->kt);
  desc->d_keys = t->d_keys;
  desc->d_offsets = t->d_offsets;
  desc->d_part_offsets = t->d_part_offsets;
  desc->d_bucket_base = t->d_bucket_base;
  desc->probe_count_bytes = t->has_long ? 4u : 1u;
  desc->reserved = 0;
  return HG_OK;
}

hg_status hg_table_export(const hg_table* table, uint32_t* d_part_offsets, uint32_t* d_bucket_base,
                          uint32_t* d_offsets, void* d_keys, hipStream_t stream) {
  if (table == nullptr) return fail(HG_ERR_INVALID_ARG, "null table");
  hg_table_desc d;
  hg_status st = hg_table_info(table, &d);
  if (st != HG_OK) return st;
  const size_t small = sizeof(uint32_t) * (table->P + 1);
  if (d_part_offsets)
    HG_TRY(hipMemcpyAsync(d_part_offsets, table->d_part_offsets, small, hipMemcpyDeviceToDevice, stream),
           "copy part_offsets");
  if (d_bucket_base)
    HG_TRY(hipMemcpyAsync(d_bucket_base, table->d_bucket_base, small, hipMemcpyDeviceToDevice, stream),
           "copy bucket_base");
  if (d_offsets)
    HG_TRY(hipMemcpyAsync(d_offsets, table->d_offsets, sizeof(uint32_t) * (d.num_buckets + 1),
                          hipMemcpyDeviceToDevice, stream),
           "copy offsets");
  if (d_keys && table->n)
    HG_TRY(hipMemcpyAsync(d_keys, table->d_keys, key_bytes(table->kt) * table->n, hipMemcpyDeviceToDevice, stream),
           "copy keys");
  return HG_OK;
}

void hg_table_free(hg_table* table) {
  if (table == nullptr) return;
  for (const TableBlock& b : table->blocks) free_block(b, table->stream);
  delete table;
}

hg_status hg_set_allocator(hg_alloc_fn alloc, hg_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(HG_ERR_INVALID_ARG, "hg_set_allocator takes both functions or neither");
  std::lock_guard<std::mutex> lk(g_hook_mu);
  g_hook.alloc = alloc;
  g_hook.free_fn = free_fn;
  g_hook.ctx = alloc ? ctx : nullptr;
  return HG_OK;
}

hg_status hg_workspace_size(hg_op op, const hg_table* table, uint64_t n, hg_key_type kt, const hg_build_opts* opts,
                            uint32_t aux, uint64_t* workspace_bytes, uint64_t* table_bytes) {
  // Run the call itself in dry-run mode: same argument checks, same sizes,
  // nothing enqueued.  The placeholder pointers only pass the null checks.
  Measure m;
  struct Scope {
    explicit Scope(Measure* mm) : prev(t_measure) { t_measure = mm; }
    ~Scope() { t_measure = prev; }
    Measure* prev;
  } scope(&m);
  void* ph = reinterpret_cast<void*>(uintptr_t(1) << 43);
  uint32_t* ph32 = static_cast<uint32_t*>(ph);
  hg_table* t = nullptr;
  hg_status st;
  switch (op) {
    case HG_OP_BUILD: st = hg_build(ph, n, kt, opts, nullptr, &t); break;
    case HG_OP_COUNT: st = hg_count_ex(table, ph, n, ph32, aux, nullptr); break;
    case HG_OP_QUERY: st = hg_query_ex(table, ph, n, static_cast<uint8_t*>(ph), aux, nullptr); break;
    case HG_OP_BUILD_BATCHED: st = hg_build_batched(ph, n, kt, aux, ph32, opts, nullptr, &t); break;
    case HG_OP_COUNT_BATCHED: st = hg_count_batched(table, ph, n, ph32, ph32, nullptr); break;
    case HG_OP_QUERY_BATCHED: st = hg_query_batched(table, ph, n, ph32, static_cast<uint8_t*>(ph), nullptr); break;
    case HG_OP_BIN_PARTITION: st = hg_bin_partition(ph, n, kt, aux, ph, ph32, nullptr); break;
    default: return fail(HG_ERR_INVALID_ARG, "unknown op %d", static_cast<int>(op));
  }
  delete t;  // its blocks are placeholders: nothing to free
  if (st != HG_OK) return st;
  if (workspace_bytes) *workspace_bytes = m.workspace;
  if (table_bytes) *table_bytes = m.table;
  return HG_OK;
}

hg_status hg_trim_pool(uint64_t keep_bytes) {
  int dev = 0;
  HG_TRY(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_cache_mu);
  HG_TRY(cache_release(g_cache[dev], keep_bytes), "release cached blocks");
  return HG_OK;
}

const char* hg_status_string(hg_status s) {
  switch (s) {
    case HG_OK: return "HG_OK";
    case HG_ERR_INVALID_ARG: return "HG_ERR_INVALID_ARG";
    case HG_ERR_OUT_OF_MEMORY: return "HG_ERR_OUT_OF_MEMORY";
    case HG_ERR_HIP: return "HG_ERR_HIP";
    case HG_ERR_UNSUPPORTED: return "HG_ERR_UNSUPPORTED";
  }
  return "HG_ERR_UNKNOWN";
}

const char* hg_last_error(void) { return t_err.c_str(); }

hg_status hg_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return HG_OK;
}

hg_status hg_profile_only(const char* name) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_only = name != nullptr ? name : "";
  return HG_OK;
}

hg_status hg_profile_collect(void) {
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs.swap(g_pending);
  }
  hg_status st = HG_OK;
  for (const ProfRec& r : recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (e != hipSuccess) {
      st = fail_hip(e, "profile event");
    } else {
      auto& tot = g_totals[r.name];
      tot.first += 1;
      tot.second += ms;
    }
    g_events.push_back(r.a);
    g_events.push_back(r.b);
  }
  return st;
}

int hg_profile_read(const char** names, uint64_t* launches, double* total_ms, int cap) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int i = 0;
  for (const auto& kv : g_totals) {
    if (i < cap) {
      if (names) names[i] = kv.first.c_str();
      if (launches) launches[i] = kv.second.first;
      if (total_ms) total_ms[i] = kv.second.second;
    }
    ++i;
  }
  return i;
}

void hg_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_totals.clear();
}

}  // extern "C"
