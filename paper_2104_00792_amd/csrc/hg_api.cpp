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
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hg_internal.h"

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
  std::mutex mu;
  bool have_num_buckets;
  uint64_t num_buckets;
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

// ------------------------------------------------------------ memory pool
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;

hipError_t pool_for(int dev, hipMemPool_t* out) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pools.find(dev);
  if (it != g_pools.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipMemPoolProps props = {};
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t pool;
  hipError_t e = hipMemPoolCreate(&pool, &props);
  if (e != hipSuccess) return e;
  uint64_t keep = UINT64_MAX;  // keep freed blocks for reuse
  e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  if (e != hipSuccess) return e;
  g_pools[dev] = pool;
  *out = pool;
  return hipSuccess;
}

// Allocations of one call; frees everything still owned on destruction.
class Allocs {
 public:
  explicit Allocs(hipStream_t s) : s_(s) {}
  ~Allocs() {
    for (void* p : owned_) (void)hipFreeAsync(p, s_);
  }
  hipError_t get(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipMemPool_t pool;
    e = pool_for(dev, &pool);
    if (e != hipSuccess) return e;
    e = hipMallocFromPoolAsync(p, bytes, pool, s_);
    if (e == hipSuccess) owned_.push_back(*p);
    return e;
  }
  // Stop owning p (it now belongs to a table).
  void release(void* p) {
    for (auto& q : owned_)
      if (q == p) q = nullptr;
    std::vector<void*> keep;
    for (void* q : owned_)
      if (q) keep.push_back(q);
    owned_.swap(keep);
  }

 private:
  hipStream_t s_;
  std::vector<void*> owned_;
};

// -------------------------------------------------------------- profiling
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_pending;
std::vector<hipEvent_t> g_events;
std::map<std::string, std::pair<uint64_t, double>> g_totals;

hipEvent_t take_event() {
  if (!g_events.empty()) {
    hipEvent_t e = g_events.back();
    g_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t s) : name_(name), s_(s) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
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
      _e = (call);                                                          \
    }                                                                       \
    if (_e != hipSuccess) return fail_hip(_e, name);                        \
    if (debug_sync()) {                                                     \
      _e = hipStreamSynchronize(stream);                                    \
      std::fprintf(stderr, "[hg] %s -> %s\n", name, hipGetErrorString(_e)); \
      if (_e != hipSuccess) return fail_hip(_e, name);                      \
    }                                                                       \
  } while (0)

#define HG_TRY(expr, what)                          \
  do {                                              \
    hipError_t _e = (expr);                         \
    if (_e != hipSuccess) return fail_hip(_e, what); \
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

hg_status probe(const hg_table* t, const void* d_queries, uint64_t q, void* d_out, bool count, hipStream_t s) {
  if (t == nullptr) return fail(HG_ERR_INVALID_ARG, "null table");
  if (q >= (1ull << 32)) return fail(HG_ERR_INVALID_ARG, "q = %llu is not below 2^32", (unsigned long long)q);
  if (q > 0 && (d_queries == nullptr || d_out == nullptr)) return fail(HG_ERR_INVALID_ARG, "null queries or output");
  if (q == 0) return HG_OK;
  HG_LAUNCH(count ? "probe_count" : "probe_found", s,
            hg::launch_probe(t->kt, count, t->d_keys, t->d_offsets, t->d_desc, t->log2P, t->P, d_queries,
                             static_cast<uint32_t>(q), d_out, s));
  return HG_OK;
}

}  // namespace

extern "C" {

hg_status hg_build(const void* d_keys, uint64_t n, hg_key_type kt, const hg_build_opts* opts, hipStream_t stream,
                   hg_table** out) {
  if (out == nullptr || opts == nullptr) return fail(HG_ERR_INVALID_ARG, "null opts or out");
  hg_status st = check_n_P(n, kt, opts->P);
  if (st != HG_OK) return st;
  if (n > 0 && d_keys == nullptr) return fail(HG_ERR_INVALID_ARG, "null keys");
  if (opts->reserved0 != 0) return fail(HG_ERR_INVALID_ARG, "reserved field is not 0");
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

  const uint32_t n32 = static_cast<uint32_t>(n);
  const uint32_t log2P = log2_of(P);
  const size_t ks = key_bytes(kt);
  const uint32_t num_tiles = hg::div_up(n, hg::kTileKeys);
  int device = 0;
  HG_TRY(hipGetDevice(&device), "hipGetDevice");

  Allocs mem(stream);
  void *keys_out = nullptr, *offsets = nullptr, *meta = nullptr;
  const size_t meta_bytes = 2 * sizeof(uint32_t) * (P + 1) + 8 + sizeof(hg::PartDesc) * P;
  HG_TRY(mem.get(&keys_out, n * ks), "allocate table keys");
  HG_TRY(mem.get(&offsets, (bound + 1) * sizeof(uint32_t)), "allocate table offsets");
  HG_TRY(mem.get(&meta, meta_bytes), "allocate table metadata");
  uint32_t* po = static_cast<uint32_t*>(meta);
  uint32_t* bb = po + (P + 1);
  uintptr_t dp = reinterpret_cast<uintptr_t>(bb + (P + 1));
  dp = (dp + 7) & ~static_cast<uintptr_t>(7);
  hg::PartDesc* desc = reinterpret_cast<hg::PartDesc*>(dp);

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
              hg::launch_layout(static_cast<uint32_t*>(tile_counts), num_tiles, P, n32, opts->ratio_num,
                                opts->ratio_den, 0, po, bb, desc, stream));
    src = buffer;
  } else {
    HG_LAUNCH("layout", stream,
              hg::launch_layout(nullptr, 0, 1, n32, opts->ratio_num, opts->ratio_den,
                                plain_V ? opts->num_buckets : 0, po, bb, desc, stream));
  }

  uint32_t* offs = static_cast<uint32_t*>(offsets);
  HG_LAUNCH("zero_counts", stream, hg::launch_fill_u32(offs, bound + 1, 0u, stream));
  HG_LAUNCH("bucket_hist", stream, hg::launch_hist(kt, src, n32, log2P, P, desc, offs + 1, stream));
  HG_LAUNCH("bucket_scan", stream,
            hg::launch_scan_exclusive(offs + 1, bb + P, bound, static_cast<uint32_t*>(bsums), stream));
  HG_LAUNCH("bucket_scatter", stream, hg::launch_scatter(kt, src, n32, log2P, P, desc, offs + 1, keys_out, stream));

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
  t->have_num_buckets = false;
  t->num_buckets = 0;
  mem.release(keys_out);
  mem.release(offsets);
  mem.release(meta);
  *out = t;
  return HG_OK;
}

hg_status hg_count(const hg_table* table, const void* d_queries, uint64_t q, uint32_t* d_counts, hipStream_t stream) {
  return probe(table, d_queries, q, d_counts, true, stream);
}

hg_status hg_query(const hg_table* table, const void* d_queries, uint64_t q, uint8_t* d_found, hipStream_t stream) {
  return probe(table, d_queries, q, d_found, false, stream);
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
      uint32_t nb = 0;
      HG_TRY(hipMemcpyAsync(&nb, t->d_bucket_base + t->P, sizeof(nb), hipMemcpyDeviceToHost, t->stream),
             "read bucket count");
      HG_TRY(hipStreamSynchronize(t->stream), "wait for build");
      t->num_buckets = nb;
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
  if (table->d_keys) (void)hipFreeAsync(table->d_keys, table->stream);
  if (table->d_offsets) (void)hipFreeAsync(table->d_offsets, table->stream);
  if (table->d_meta) (void)hipFreeAsync(table->d_meta, table->stream);
  delete table;
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
