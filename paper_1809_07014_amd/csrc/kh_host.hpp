// Host-side internals shared by the C ABI (kh_api.hip) and the serving
// engine (kh_server.hip): error reporting, the context's device memory pool,
// the context and table objects, and the table-finishing pipeline.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>

#include "kh_internal.hpp"
#include "kmerhip.h"

namespace kh {

// ------------------------------------------------------------- errors ----

inline thread_local std::string g_err;

inline int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                      \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess)                                                  \
      return fail(KH_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define KH_TRY(expr)          \
  do {                        \
    int r_ = (expr);          \
    if (r_ != KH_OK) return r_; \
  } while (0)

// --------------------------------------------------------------- pool ----

// Blocks left by destroyed contexts, kept per device for the next context
// there: allocating again right after freeing tens of GB has been measured
// to stall for seconds, where taking a kept block costs nothing.
constexpr int kMaxDevices = 64;
struct DeviceCache {
  std::mutex mu;
  std::multimap<uint64_t, void*> blocks;
  // Take a kept block of at least `bytes` and at most twice that; its size
  // goes to *size.
  void* take(uint64_t bytes, uint64_t* size) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = blocks.lower_bound(bytes);
    if (it == blocks.end() || it->first > 2 * bytes + (8ull << 20)) return nullptr;
    void* p = it->second;
    *size = it->first;
    blocks.erase(it);
    return p;
  }
  void give(uint64_t bytes, void* p) {
    std::lock_guard<std::mutex> lk(mu);
    blocks.emplace(bytes, p);
  }
  void release() {  // the device's current device must be this one
    std::lock_guard<std::mutex> lk(mu);
    for (auto& kv : blocks) (void)hipFree(kv.second);
    blocks.clear();
  }
  bool empty() {
    std::lock_guard<std::mutex> lk(mu);
    return blocks.empty();
  }
};
DeviceCache& device_cache(int device);

// Caching pool of device blocks owned by one context.  Blocks are reused
// best-fit (a cached block is taken if it is at most twice the request),
// first from the context's own cache, then from the device's; when the
// budget would be exceeded, the context's cached blocks are returned to the
// device first.  Reuse is ordered by the context's stream: every public call
// finishes its device work before returning.
struct Pool {
  std::recursive_mutex mu;  // tables may be freed from another thread
  int device = 0;
  uint64_t budget = 0;
  // the caller's allocator (both set) or hipMalloc/hipFree (both null)
  kh_alloc_fn alloc_fn = nullptr;
  kh_free_fn free_fn = nullptr;
  void* user = nullptr;
  uint64_t held = 0;
  uint64_t peak = 0;
  uint64_t cached_bytes = 0;  // of `held`: blocks free for reuse
  uint64_t n_alloc = 0;  // device allocations (hipMalloc or the caller's)
  double alloc_s = 0;    // seconds spent in them
  std::multimap<uint64_t, void*> cached;
  std::unordered_map<void*, uint64_t> size_of;

  // Arena mode (arena != nullptr; the no-allocation entry point): blocks are
  // carved from one fixed device range in stack order and nothing is ever
  // allocated or freed.  A block given back is reclaimed once every block
  // carved after it has been given back too (callers release in reverse
  // order of allocation, as scoped buffers do).
  static constexpr int kArenaDepth = 64;
  uint8_t* arena = nullptr;
  uint64_t arena_size = 0, arena_used = 0;
  int arena_top = 0;
  uint64_t arena_off[kArenaDepth] = {};
  void* arena_blk[kArenaDepth] = {};
  bool arena_gone[kArenaDepth] = {};

  // Bytes an arena block of `bytes` takes (256-byte granules).
  static uint64_t arena_round(uint64_t b) { return (std::max<uint64_t>(b, 1) + 255) / 256 * 256; }
  uint64_t arena_free() const { return arena_size - arena_used; }

  int arena_get(void** out, uint64_t bytes) {
    bytes = arena_round(bytes);
    if (arena_top == kArenaDepth || bytes > arena_size - arena_used)
      return fail(KH_ENOMEM, "the no-allocation scratch (%llu bytes) cannot hold a block "
                             "of %llu bytes (%llu in use)",
                  (unsigned long long)arena_size, (unsigned long long)bytes,
                  (unsigned long long)arena_used);
    arena_off[arena_top] = arena_used;
    arena_blk[arena_top] = arena + arena_used;
    arena_gone[arena_top] = false;
    ++arena_top;
    *out = arena + arena_used;
    arena_used += bytes;
    held = arena_used;
    peak = std::max(peak, held);
    return KH_OK;
  }
  void arena_put(void* p) {
    for (int i = arena_top - 1; i >= 0; --i)
      if (arena_blk[i] == p) {
        arena_gone[i] = true;
        break;
      }
    while (arena_top > 0 && arena_gone[arena_top - 1]) {
      --arena_top;
      arena_used = arena_off[arena_top];
    }
    held = arena_used;
  }

  static uint64_t round(uint64_t b) {
    if (b < 256) b = 256;
    const uint64_t g = b >= (2ull << 20) ? (2ull << 20) : 256ull;
    return (b + g - 1) / g * g;
  }

  hipError_t raw_alloc(void** p, uint64_t bytes) {
    if (!alloc_fn) return hipMalloc(p, bytes);
    *p = alloc_fn(bytes, device, user);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  void raw_free(void* p, uint64_t bytes) {
    if (free_fn)
      free_fn(p, bytes, device, user);
    else
      (void)hipFree(p);
  }

  void drop_cached() {
    std::lock_guard<std::recursive_mutex> lk(mu);
    // a free block may still be named by queued work of this context; the
    // caller's allocator may hand it out on another stream at once, so the
    // device finishes first (hipFree waits by itself)
    if (free_fn && !cached.empty()) (void)hipDeviceSynchronize();
    for (auto& kv : cached) {
      raw_free(kv.second, kv.first);
      held -= kv.first;
      size_of.erase(kv.second);
    }
    cached.clear();
    cached_bytes = 0;
  }

  int get(void** out, uint64_t bytes) {
    std::lock_guard<std::recursive_mutex> lk(mu);
    if (arena) return arena_get(out, bytes);
    bytes = round(bytes);
    auto it = cached.lower_bound(bytes);
    if (it != cached.end() && it->first <= 2 * bytes + (8ull << 20)) {
      *out = it->second;
      cached_bytes -= it->first;
      cached.erase(it);
      return KH_OK;
    }
    if (budget && held + bytes > budget) drop_cached();
    if (budget && held + bytes > budget)
      return fail(KH_ENOMEM, "device budget exceeded: need %llu more bytes, "
                             "hold %llu of %llu",
                  (unsigned long long)bytes, (unsigned long long)held,
                  (unsigned long long)budget);
    void* p = nullptr;
    uint64_t sz = 0;
    if (void* q = alloc_fn ? nullptr : device_cache(device).take(bytes, &sz)) {
      // left by a destroyed context
      if (budget && held + sz > budget) {
        device_cache(device).give(sz, q);  // too big for the budget: allocate
      } else {
        size_of[q] = sz;
        held += sz;
        peak = std::max(peak, held);
        *out = q;
        return KH_OK;
      }
    }
    const auto t0 = std::chrono::steady_clock::now();
    {  // kept blocks that fit no request give way before the device fills up
      DeviceCache& dc = device_cache(device);
      size_t free_b = 0, total_b = 0;
      if (!alloc_fn && !dc.empty() && hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
          free_b < bytes + (4ull << 30))
        dc.release();
    }
    hipError_t e = raw_alloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      drop_cached();
      if (!alloc_fn) device_cache(device).release();
      e = raw_alloc(&p, bytes);
    }
    alloc_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    ++n_alloc;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(KH_ENOMEM, "device allocation of %llu bytes failed: %s",
                  (unsigned long long)bytes, hipGetErrorString(e));
    }
    size_of[p] = bytes;
    held += bytes;
    peak = std::max(peak, held);
    *out = p;
    return KH_OK;
  }

  void put(void* p) {
    std::lock_guard<std::recursive_mutex> lk(mu);
    if (!p) return;
    if (arena) {
      arena_put(p);
      return;
    }
    auto it = size_of.find(p);
    if (it == size_of.end()) return;
    cached.emplace(it->second, p);
    cached_bytes += it->second;
  }

  // Hand every block to the device's cache, or back to the caller's
  // allocator (the context is going away and its device work has finished).
  void release_all() {
    std::lock_guard<std::recursive_mutex> lk(mu);
    DeviceCache& dc = device_cache(device);
    for (auto& kv : size_of) {
      if (free_fn)
        raw_free(kv.first, kv.second);
      else
        dc.give(kv.second, kv.first);
    }
    cached.clear();
    size_of.clear();
    held = 0;
    cached_bytes = 0;
  }
};

// Scoped pool block.
template <typename T>
struct Buf {
  Pool* pool = nullptr;
  T* p = nullptr;
  Buf() = default;
  explicit Buf(Pool* pl) : pool(pl) {}
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  ~Buf() { reset(); }
  int alloc(uint64_t count) {
    reset();
    void* v = nullptr;
    KH_TRY(pool->get(&v, std::max<uint64_t>(count, 1) * sizeof(T)));
    p = static_cast<T*>(v);
    return KH_OK;
  }
  void reset() {
    if (p && pool) pool->put(p);
    p = nullptr;
  }
  T* release() {
    T* r = p;
    p = nullptr;
    return r;
  }
};

// ------------------------------------------------------------ objects ----

enum { kTimeEvents = 12 };  // start/end pairs: pack, Bloom, count, classify, sort, gather
enum { kMaxK = 8, kStats = 12 };
}  // namespace kh

// The C ABI's opaque objects (declared in kmerhip.h at global scope).

struct kh_ctx {
  int device = 0;
  int cus = 256;                      // compute units of the device
  kh::Pool pool;
  unsigned long long* ctr = nullptr;  // kCtrCount counters
  int timing = 0;
  hipEvent_t ev[kh::kTimeEvents] = {};
  float last_ms[6] = {0, 0, 0, 0, 0, 0};
  uint64_t last_stats[kh::kStats] = {};
  int cur_k = 0;                      // index of the k being counted
  float k_ms[kh::kMaxK][6] = {};      // per-k phase times of the last call
  uint64_t k_stats[kh::kMaxK][kh::kStats] = {};
  std::unordered_set<kh_table*> live;  // tables whose rows live in `pool`
  // batched multi-k pipeline
  unsigned long long* kctr = nullptr;    // kMaxK blocks of kCtrCount counters
  hipStream_t side = nullptr;            // per-k tails overlap the next passes
  hipStream_t capture = nullptr;         // graph capture of the counting passes
  hipEvent_t copy_ev = nullptr;          // a streamed upload's chunk has arrived
  hipEvent_t kev[kh::kMaxK][2] = {};     // start/end of each counting pass
  hipGraphExec_t graph_exec = nullptr;   // counting passes of the last call
  int last_graphed = 0;                  // the last batched call replayed it
  kh_tuning tune{};   // free parameters (kh_default_tuning, kh_set_tuning)
  std::unordered_set<kh_contigs*> live_contigs;  // contigs whose data live in `pool`
};

struct kh_table {
  kh_ctx* ctx = nullptr;
  uint32_t k = 0, W = 0;
  uint64_t serial = 0;  // unique per table in the process (make_table)
  int64_t n_rows = 0;
  uint64_t n_windows = 0;
  uint64_t* keys = nullptr;
  uint32_t* counts = nullptr;
  uint32_t* ext = nullptr;
  uint8_t* codes = nullptr;
  // Rows written to the caller's device buffers instead of the pool (the
  // no-allocation entry point): enabled when dst_cap >= 0, which is the
  // number of rows they hold.
  uint64_t* dst_keys = nullptr;
  uint32_t* dst_counts = nullptr;
  uint32_t* dst_ext = nullptr;
  uint8_t* dst_codes = nullptr;
  int64_t dst_cap = -1;
};

struct kh_contigs {
  kh_ctx* ctx = nullptr;
  uint32_t k = 0;
  int64_t n_contigs = 0, total_bases = 0;
  char* seq = nullptr;        // total_bases ASCII
  int64_t* offsets = nullptr;  // n_contigs + 1
  int64_t* n_kmers = nullptr;
  uint64_t* depth = nullptr;
  uint8_t* cycle = nullptr;
  // Contigs walked from a table: the serial of that table, its row count and
  // the contig of every row (row order).  Pruned contigs keep none of these.
  uint64_t source = 0;
  int64_t n_rows = 0;
  uint32_t* row_contig = nullptr;
  int rounds = 0;             // pointer-jumping rounds run (both passes)
  int64_t cycle_kmers = 0;    // k-mers on cycles
};



namespace kh {

// Count pipeline pieces used by both the one-shot calls and serving.
using RecountFn = std::function<int(HeavyEntry* heavy, uint32_t* index,
                                    uint32_t mask)>;
int make_table(kh_ctx* ctx, uint32_t k, kh_table** out);
// Reads (device) copied in `order` (device read indices) into o_seq, o_qual
// (offsets[n_reads] bytes) and o_off (n_reads + 1); KH_EINVAL if order is
// not a permutation.
int gather_reads_ordered(Pool* pool, const uint8_t* seq, const uint8_t* qual,
                         const int64_t* offsets, int64_t n_reads, const int64_t* order,
                         uint8_t* o_seq, uint8_t* o_qual, int64_t* o_off, hipStream_t s);
// Reads (device, n bases) copied in the order of their minimizers into
// o_seq, o_qual, o_off; KH_EINVAL for bad offsets.
int reorder_by_minimizer(Pool* pool, const uint8_t* seq, const uint8_t* qual,
                         const int64_t* offsets, int64_t n_reads, int64_t n, hipStream_t s,
                         uint8_t* o_seq, uint8_t* o_qual, int64_t* o_off);
int read_ctr(kh_ctx* ctx, hipStream_t s, uint64_t (&c)[kCtrCount]);
int read_ctr_at(const unsigned long long* ctr, hipStream_t s,
                uint64_t (&c)[kCtrCount]);
int finish_rows(kh_ctx* ctx, unsigned long long* ctr, uint8_t* table,
                uint64_t cap, const kh_params& p, const RecountFn& recount,
                hipStream_t s, kh_table* t);
int check_params(const kh_params* p);
// Pack a read set and count one k into an existing table object (whose rows
// may go to the caller's buffers, kh_table::dst_cap); no streamed upload.
int count_into(kh_ctx* ctx, const kh_reads* reads, const kh_params& p, hipStream_t s,
               kh_table* t);

}  // namespace kh

// Contigs of a destroyed context lose their data (kh_destroy).
void kh_orphan_contigs(kh_ctx* ctx);

// Exclusive prefix sum of n uint64 values on the stream; *total (device)
// receives the sum of all.
int kh_scan_exclusive_u64(kh::Pool* pool, const uint64_t* in, uint64_t* out, int64_t n,
                          uint64_t* total, hipStream_t s);
