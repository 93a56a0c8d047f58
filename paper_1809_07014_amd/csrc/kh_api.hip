// Host side of the C ABI declared in include/kmerhip.h: context, device
// memory pool, parameter validation, capacity planning and the pipeline
// pack -> [Bloom pass A] -> count pass -> classify/compact -> sort -> gather.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <numeric>
#include <vector>

#include "kh_host.hpp"

using namespace kh;

// Device planes of one packed read set.
struct Packed {
  Buf<uint64_t> bases, hq, bad, st;
  Buf<uint8_t> seq_copy, qual_copy, seq_sorted, qual_sorted;
  Buf<int64_t> off_copy, off_sorted;
  int64_t n = 0, n_reads = 0, base_words = 0, plane_words = 0;
  // Streamed upload of host reads: bases [0, packed) are on the device and
  // packed; the rest is copied and packed in chunks by the caller of
  // pack_reads (overlapping the copies with the Bloom pass), or at once by
  // finish_pack.
  PackArgs pa{};
  const uint8_t* host_seq = nullptr;
  const uint8_t* host_qual = nullptr;
  int64_t packed = 0;
  // The stream a streamed upload copies on, once copies may be in flight:
  // the buffers go back to the pool only after it has drained, so that no
  // later owner of a block (or of the caller's host buffers) races a copy
  // left behind by an early return.
  hipStream_t copy_stream = nullptr;
  explicit Packed(Pool* p)
      : bases(p), hq(p), bad(p), st(p), seq_copy(p), qual_copy(p), seq_sorted(p),
        qual_sorted(p), off_copy(p), off_sorted(p) {}
  ~Packed() {
    if (copy_stream) (void)hipStreamSynchronize(copy_stream);
  }
};

// ------------------------------------------------------------ helpers ----

extern "C" void kh_default_params(kh_params* p, uint32_t k) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->k = k;
  p->min_count = 2;
  p->qual_offset = 33;
  p->qual_cutoff = 20;
  p->t_min_ext = 2;
  p->t_base = 1;
  p->err_ppm = 5000;
  p->use_bloom = 0;
  p->bloom_bits = 0;
  p->load_factor = 0.0f;
  p->owner_shards = 0;
  p->owner = 0;
}

static uint64_t host_mix(uint64_t z) {  // SplitMix64 output function
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

extern "C" uint32_t kh_owner_of(const uint64_t* key, uint32_t W, uint32_t shards) {
  if (!key || shards <= 1) return 0;
  uint64_t h = 0;
  for (uint32_t j = 0; j < W; ++j) h = host_mix(h ^ key[j]);
  return (uint32_t)(h % shards);
}

extern "C" const char* kh_last_error(void) { return g_err.c_str(); }

int kh::check_params(const kh_params* p) {
  if (!p) return fail(KH_EINVAL, "params is NULL");
  if (p->k < 1 || p->k > 127 || (p->k % 2) == 0)
    return fail(KH_EINVAL, "k must be odd and in 1..127 (got %u)", p->k);
  if (p->min_count < 1 || p->min_count > kHeavyCount)
    return fail(KH_EINVAL, "min_count must be in 1..%u", kHeavyCount);
  if (p->use_bloom && p->min_count < 2)
    return fail(KH_EINVAL, "the Bloom pass needs min_count >= 2");
  if (p->qual_offset > 255) return fail(KH_EINVAL, "qual_offset > 255");
  if (!(p->load_factor >= 0.0f && p->load_factor < 0.95f))
    return fail(KH_EINVAL, "load_factor must be in [0, 0.95)");
  if (p->bloom_bits > 64) return fail(KH_EINVAL, "bloom_bits must be in 0..64");
  if (p->owner_shards > 1 && p->owner >= p->owner_shards)
    return fail(KH_EINVAL, "owner %u is not below owner_shards %u", p->owner, p->owner_shards);
  return KH_OK;
}

static int set_device(kh_ctx* ctx) {
  HIP_TRY(hipSetDevice(ctx->device));
  return KH_OK;
}

static void mark(kh_ctx* ctx, int i, hipStream_t s) {
  if (ctx->timing) (void)hipEventRecord(ctx->ev[i], s);
}

// Add the measured phase durations (event pairs 1..5) after a synchronise.
static void accumulate_phases(kh_ctx* ctx, int first, int last) {
  if (!ctx->timing) return;
  for (int ph = first; ph <= last; ++ph) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ctx->ev[2 * ph], ctx->ev[2 * ph + 1]) != hipSuccess) {
      (void)hipGetLastError();
      ms = 0.0f;
    }
    ctx->last_ms[ph] += ms;
    if (ctx->cur_k < kMaxK) ctx->k_ms[ctx->cur_k][ph] += ms;
  }
}

// Bases per chunk of a streamed upload (a multiple of 64 and of the tile):
// 128 Mi, or KMERHIP_STREAM_CHUNK rounded up to whole tiles (a testing hook
// that lets small read sets take the streamed path).
static int64_t stream_chunk_bases() {
  const char* e = std::getenv("KMERHIP_STREAM_CHUNK");
  if (!e) return 128ll << 20;
  const int64_t v = std::max<int64_t>(1, std::strtoll(e, nullptr, 10));
  return (v + kTile - 1) / kTile * kTile;
}

// Copy bases and qualities [p0, p1) of streamed host reads to the device on
// `copy` and pack them on `s` (which waits for the copy).
static int stream_chunk(kh_ctx* ctx, Packed& pk, int64_t p0, int64_t p1, hipStream_t s,
                        hipStream_t copy) {
  HIP_TRY(hipMemcpyAsync(pk.seq_copy.p + p0, pk.host_seq + p0, p1 - p0,
                         hipMemcpyHostToDevice, copy));
  HIP_TRY(hipMemcpyAsync(pk.qual_copy.p + p0, pk.host_qual + p0, p1 - p0,
                         hipMemcpyHostToDevice, copy));
  HIP_TRY(hipEventRecord(ctx->copy_ev, copy));
  HIP_TRY(hipStreamWaitEvent(s, ctx->copy_ev, 0));
  launch_pack_range(pk.pa, p0, p1, s);
  HIP_TRY(hipGetLastError());
  pk.packed = p1;
  return KH_OK;
}

// Copy and pack whatever a streamed upload has not yet packed.
static int finish_pack(kh_ctx* ctx, Packed& pk, hipStream_t s) {
  if (pk.packed < pk.n) KH_TRY(stream_chunk(ctx, pk, pk.packed, pk.n, s, ctx->side));
  return KH_OK;
}

// Upload (if needed) and pack a read set into device bit planes.
// allow_stream: host reads may be left for the caller to upload in chunks
// (Packed::packed says how far they are).
static int pack_reads(kh_ctx* ctx, const kh_reads* r, const kh_params& p,
                      hipStream_t s, Packed& pk, bool allow_stream = false) {
  if (!r) return fail(KH_EINVAL, "reads is NULL");
  if (r->n_reads < 0) return fail(KH_EINVAL, "n_reads < 0");
  pk.n_reads = r->n_reads;
  if (r->n_reads > 0 && !r->offsets) return fail(KH_EINVAL, "offsets is NULL");
  int64_t n = 0;
  if (r->n_reads > 0) {
    if (r->on_device) {
      int64_t ends[1];
      HIP_TRY(hipMemcpyAsync(ends, r->offsets + r->n_reads, sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      n = ends[0];
    } else {
      if (r->offsets[0] != 0) return fail(KH_EINVAL, "offsets[0] must be 0");
      for (int64_t i = 0; i < r->n_reads; ++i)
        if (r->offsets[i + 1] < r->offsets[i])
          return fail(KH_EINVAL, "offsets decrease at read %lld", (long long)i);
      n = r->offsets[r->n_reads];
    }
  }
  if (n < 0) return fail(KH_EINVAL, "offsets[n_reads] < 0");
  if (n > 0 && (!r->seq || !r->qual)) return fail(KH_EINVAL, "seq or qual is NULL");
  pk.n = n;
  pk.packed = n;
  if (n == 0) return KH_OK;

  const uint8_t* seq = reinterpret_cast<const uint8_t*>(r->seq);
  const uint8_t* qual = reinterpret_cast<const uint8_t*>(r->qual);
  const int64_t* off = r->offsets;
  const bool streamed = !r->on_device && allow_stream && !ctx->tune.aggregate &&
                        n >= 2 * stream_chunk_bases();
  if (streamed) {  // offsets now; bases and qualities chunk by chunk later
    KH_TRY(pk.seq_copy.alloc((uint64_t)n));
    KH_TRY(pk.qual_copy.alloc((uint64_t)n));
    KH_TRY(pk.off_copy.alloc((uint64_t)r->n_reads + 1));
    HIP_TRY(hipMemcpyAsync(pk.off_copy.p, off, sizeof(int64_t) * (r->n_reads + 1),
                           hipMemcpyHostToDevice, s));
    // the copy stream starts after the caller's stream reaches this point:
    // a block the caller's allocator hands out may have been freed on that
    // stream while its earlier work still reads it
    HIP_TRY(hipEventRecord(ctx->copy_ev, s));
    HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->copy_ev, 0));
    pk.copy_stream = ctx->side;
    pk.host_seq = seq;
    pk.host_qual = qual;
    pk.packed = 0;
    seq = pk.seq_copy.p;
    qual = pk.qual_copy.p;
    off = pk.off_copy.p;
  } else if (!r->on_device) {
    KH_TRY(pk.seq_copy.alloc((uint64_t)n));
    KH_TRY(pk.qual_copy.alloc((uint64_t)n));
    KH_TRY(pk.off_copy.alloc((uint64_t)r->n_reads + 1));
    HIP_TRY(hipMemcpyAsync(pk.seq_copy.p, seq, n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(pk.qual_copy.p, qual, n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(pk.off_copy.p, off, sizeof(int64_t) * (r->n_reads + 1),
                           hipMemcpyHostToDevice, s));
    seq = pk.seq_copy.p;
    qual = pk.qual_copy.p;
    off = pk.off_copy.p;
  }
  if (ctx->tune.aggregate && r->n_reads > 1) {
    // reads in minimizer order: a k-mer's occurrences land in nearby tiles,
    // where the aggregating counting pass merges them
    KH_TRY(pk.seq_sorted.alloc((uint64_t)n));
    KH_TRY(pk.qual_sorted.alloc((uint64_t)n));
    KH_TRY(pk.off_sorted.alloc((uint64_t)r->n_reads + 1));
    KH_TRY(reorder_by_minimizer(&ctx->pool, seq, qual, off, r->n_reads, n, s,
                                pk.seq_sorted.p, pk.qual_sorted.p, pk.off_sorted.p));
    pk.seq_copy.reset();
    pk.qual_copy.reset();
    seq = pk.seq_sorted.p;
    qual = pk.qual_sorted.p;
    off = pk.off_sorted.p;
  }
  pk.base_words = (n + 31) / 32 + 2;
  pk.plane_words = (n + 63) / 64 + 2;
  KH_TRY(pk.bases.alloc((uint64_t)pk.base_words));
  KH_TRY(pk.hq.alloc((uint64_t)pk.plane_words));
  KH_TRY(pk.bad.alloc((uint64_t)pk.plane_words));
  KH_TRY(pk.st.alloc((uint64_t)pk.plane_words));
  // pad words beyond n: no base, not a start
  launch_fill_u64(pk.bases.p, (uint64_t)pk.base_words, 0ull, s);
  launch_fill_u64(pk.hq.p, (uint64_t)pk.plane_words, 0ull, s);
  launch_fill_u64(pk.bad.p, (uint64_t)pk.plane_words, ~0ull, s);
  PackArgs a{};
  a.seq = seq;
  a.qual = qual;
  a.offsets = off;
  a.n_reads = r->n_reads;
  a.n = n;
  a.qual_offset = (int)p.qual_offset;
  a.qual_cutoff = (int)p.qual_cutoff;
  a.bases = pk.bases.p;
  a.hq = pk.hq.p;
  a.bad = pk.bad.p;
  a.st = pk.st.p;
  a.plane_words = pk.plane_words;
  a.ctr = ctx->ctr;
  launch_fill_u64(reinterpret_cast<uint64_t*>(ctx->ctr), kCtrCount, 0ull, s);
  pk.pa = a;
  if (streamed)
    launch_mark_starts(a, s);
  else
    launch_pack(a, s);
  HIP_TRY(hipGetLastError());
  return KH_OK;
}

int kh::read_ctr_at(const unsigned long long* ctr, hipStream_t s,
                    uint64_t (&c)[kCtrCount]) {
  HIP_TRY(hipMemcpyAsync(c, ctr, sizeof(uint64_t) * kCtrCount,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return KH_OK;
}

int kh::read_ctr(kh_ctx* ctx, hipStream_t s, uint64_t (&c)[kCtrCount]) {
  return read_ctr_at(ctx->ctr, s, c);
}

int kh::make_table(kh_ctx* ctx, uint32_t k, kh_table** out) {
  kh_table* t = new (std::nothrow) kh_table();
  if (!t) return fail(KH_ENOMEM, "host allocation failed");
  static std::atomic<uint64_t> next_serial{1};
  t->ctx = ctx;
  t->k = k;
  t->W = (k + 31) / 32;
  t->serial = next_serial.fetch_add(1);
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->pool.mu);
    ctx->live.insert(t);
  }
  *out = t;
  return KH_OK;
}

// Turn a filled table into sorted rows: classify + compact, exact recount of
// heavy k-mers, sort by key prefix (+ full-key order of equal prefixes),
// gather keys / counts / tallies / codes.  Events 6..11 time the phases.
int kh::finish_rows(kh_ctx* ctx, unsigned long long* ctr, uint8_t* table,
                    uint64_t cap, const kh_params& p, const RecountFn& recount,
                    hipStream_t s, kh_table* t) {
  const uint32_t k = p.k;
  const int W = (int)(k + 31) / 32;
  Pool* pool = &ctx->pool;
  uint64_t c[kCtrCount];
  launch_reset_ctr(ctr, 0, s);

  Buf<uint64_t> pfx_a(pool);
  Buf<uint32_t> idx_a(pool);
  Buf<uint32_t> heavy_list(pool);
  KH_TRY(pfx_a.alloc(cap));
  KH_TRY(idx_a.alloc(cap));
  KH_TRY(heavy_list.alloc(kHeavyMax));
  ClassifyArgs ca{};
  ca.table = table;
  ca.capacity = cap;
  ca.k = k;
  ca.min_count = p.min_count;
  ca.pfx_out = pfx_a.p;
  ca.idx_out = idx_a.p;
  ca.heavy_list = heavy_list.p;
  ca.ctr = ctr;
  mark(ctx, 6, s);
  launch_classify(ca, s);
  HIP_TRY(hipGetLastError());
  mark(ctx, 7, s);
  KH_TRY(read_ctr_at(ctr, s, c));
  const int64_t rows = (int64_t)c[kCtrRows];
  if (t->dst_cap >= 0 && rows > t->dst_cap) {
    t->n_rows = rows;
    return fail(KH_EOVERFLOW, "%lld rows do not fit the %lld rows of the output buffers",
                (long long)rows, (long long)t->dst_cap);
  }

  // ---- heavy hitters: k-mers seen kHeavyCount times or more get their count
  // and tallies recounted exactly in a second streaming pass over a small
  // side table
  const uint64_t n_heavy = c[kCtrHeavy];
  if (n_heavy > kHeavyMax)
    return fail(KH_EOVERFLOW, "%llu k-mers have count >= %u (at most %u are "
                "supported per table)", (unsigned long long)n_heavy, kHeavyCount,
                kHeavyMax);
  Buf<HeavyEntry> heavy(pool);
  Buf<uint32_t> heavy_index(pool);
  if (n_heavy > 0) {
    uint32_t isize = 64;
    while (isize < 4 * n_heavy) isize <<= 1;
    KH_TRY(heavy.alloc(n_heavy));
    KH_TRY(heavy_index.alloc(isize));
    launch_fill_u64(reinterpret_cast<uint64_t*>(heavy_index.p), isize / 2, ~0ull, s);
    HeavyBuildArgs hb{};
    hb.table = table;
    hb.k = k;
    hb.heavy_list = heavy_list.p;
    hb.n_heavy = (uint32_t)n_heavy;
    hb.heavy = heavy.p;
    hb.heavy_index = heavy_index.p;
    hb.heavy_mask = isize - 1;
    launch_heavy_build(hb, s);
    KH_TRY(recount(heavy.p, heavy_index.p, isize - 1));
    HIP_TRY(hipGetLastError());
  }
  ctx->last_stats[5] = (uint64_t)rows;
  ctx->last_stats[9] = n_heavy;
  ctx->last_stats[10] = k;

  // ---- sort rows by their key prefix, order runs of equal prefixes by the
  // full key, then gather keys / counts / tallies / codes
  Buf<uint64_t> pfx_b(pool);
  Buf<uint32_t> idx_b(pool);
  Buf<uint32_t> tmp(pool);
  uint32_t* idx_sorted = idx_a.p;
  mark(ctx, 8, s);
  if (rows > 1) {
    KH_TRY(pfx_b.alloc((uint64_t)rows));
    KH_TRY(idx_b.alloc((uint64_t)rows));
    KH_TRY(tmp.alloc(sort_tmp_words(rows)));
    const int pbits = 2 * k <= 64 ? 2 * (int)k : kSortPrefixBits;
    // the segmented sort's bucket table; without it the plain LSD sort runs
    Buf<uint8_t> sortx(pool);
    if (const uint64_t sxb = seg_sort_bytes(rows, pbits))
      if (sortx.alloc(sxb) != KH_OK) sortx.reset();
    int which = 0;
    if (sort_rows(pfx_a.p, idx_a.p, pfx_b.p, idx_b.p, rows, pbits, tmp.p, sortx.p, s, &which))
      return fail(KH_EDEVICE, "row sort failed: %s", hipGetErrorString(hipGetLastError()));
    uint64_t* pfx_sorted = which ? pfx_b.p : pfx_a.p;
    idx_sorted = which ? idx_b.p : idx_a.p;
    if (2 * k > 64) {
      launch_fix_ties(pfx_sorted, idx_sorted, rows, table, k, ctr, s);
      HIP_TRY(hipGetLastError());
      KH_TRY(read_ctr_at(ctr, s, c));
      if (c[kCtrStatus] & kStatusLongTies) {
        // many keys share their top 20 bases: sort by the full key instead
        Buf<uint64_t> ka(pool), kb(pool);
        KH_TRY(ka.alloc((uint64_t)rows * W));
        KH_TRY(kb.alloc((uint64_t)rows * W));
        uint32_t* other = which ? idx_a.p : idx_b.p;
        launch_row_keys(idx_sorted, rows, table, k, ka.p, s);
        const int bits0 = 2 * (int)k - 64 * (W - 1);
        const int w2 = radix_sort(ka.p, idx_sorted, kb.p, other, rows, W, bits0,
                                  tmp.p, s);
        HIP_TRY(hipGetLastError());
        if (w2) idx_sorted = other;
        HIP_TRY(hipStreamSynchronize(s));
        ctx->last_stats[11] = 1;  // full-key sort was needed
      }
    }
    HIP_TRY(hipGetLastError());
  }
  mark(ctx, 9, s);
  Buf<uint32_t> counts(pool), ext(pool);
  Buf<uint8_t> codes(pool);
  Buf<uint64_t> keys(pool);
  const bool to_caller = t->dst_cap >= 0;
  if (!to_caller) {
    KH_TRY(keys.alloc((uint64_t)rows * W));
    KH_TRY(counts.alloc((uint64_t)rows));
    KH_TRY(ext.alloc((uint64_t)rows * 8));
    KH_TRY(codes.alloc((uint64_t)rows * 2));
  }
  GatherArgs ga{};
  ga.table = table;
  ga.heavy = heavy.p;
  ga.idx = idx_sorted;
  ga.keys = to_caller ? t->dst_keys : keys.p;
  ga.n_rows = rows;
  ga.k = k;
  ga.t_min_ext = p.t_min_ext;
  ga.t_base = p.t_base;
  ga.err_ppm = p.err_ppm;
  ga.counts = to_caller ? t->dst_counts : counts.p;
  ga.ext = to_caller ? t->dst_ext : ext.p;
  ga.codes = to_caller ? t->dst_codes : codes.p;
  mark(ctx, 10, s);
  launch_gather(ga, s);
  HIP_TRY(hipGetLastError());
  mark(ctx, 11, s);
  HIP_TRY(hipStreamSynchronize(s));

  t->n_rows = rows;
  if (!to_caller) {
    t->keys = keys.release();
    t->counts = counts.release();
    t->ext = ext.release();
    t->codes = codes.release();
  }
  return KH_OK;
}

// Does the owner-partitioned count apply?  It does whenever the tuning asks
// for it, except in arena mode (the no-allocation entry point sizes its
// scratch for the single-table layout), with the LDS-aggregating pass
// selected, or under the forced-capacity testing hook (a property of the
// single table).
static bool owned_applies(const kh_ctx* ctx) {
  return ctx->tune.partitioned && !ctx->tune.aggregate && !ctx->pool.arena &&
         !std::getenv("KMERHIP_FORCE_CAPACITY");
}

// Owner-partitioned count of one k over packed reads into t (Section II-B,
// as the paper distributes it; kh_owner.hip describes the layout): route
// every window's record to the owner of its key prefix with two streaming
// partition passes, run Bloom pass A, count pass B and classify inside each
// owner's workgroup, and copy the owners' rows to the table, sorting each
// owner's by key on the way.
// *unfit = true (and nothing counted) when some owner's keys do not fit its
// LDS table even after two finer splits: the caller then counts this k with
// the single-table path.  ctx->ctr[kCtrStatus] carries the pack stage's
// status.
static int count_owned(kh_ctx* ctx, Packed& pk, const kh_params& p, hipStream_t s,
                       kh_table* t, bool* unfit) {
  *unfit = false;
  const uint32_t k = p.k;
  const int W = (int)(k + 31) / 32;
  const int R = own_record_words(k);
  Pool* pool = &ctx->pool;
  unsigned long long* ctr = ctx->ctr;
  std::memset(ctx->last_stats, 0, sizeof ctx->last_stats);
  KH_TRY(finish_pack(ctx, pk, s));
  launch_reset_ctr(ctr, kStatusBadOffsets, s);
  if (pk.n == 0) {
    HIP_TRY(hipStreamSynchronize(s));
    return KH_OK;
  }
  const uint32_t shards = p.owner_shards > 1 ? p.owner_shards : 1;
  const int p1 = own_p1(k);  // level-1 digit: 1,024 buckets
  const int nb1 = 1 << p1;
  const int64_t n_tiles = (pk.n + 4 * kTile - 1) / (4 * kTile);  // routing tiles
  // one routing block per compute unit: each block's bucket cursors write
  // 1,024 streams, and fewer blocks keep the streams' open lines in L2
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_tiles, ctx->cus));

  // ---- level 1: bucket histogram matrix, its scan, the bucket starts
  Buf<uint32_t> h1(pool), b1(pool), part(pool);
  KH_TRY(h1.alloc((uint64_t)nb1 * grid));
  KH_TRY(b1.alloc((uint64_t)nb1));
  KH_TRY(part.alloc(scan_tmp_words((int64_t)nb1 * grid)));
  OwnRouteArgs ra{};
  ra.bases = pk.bases.p;
  ra.hq = pk.hq.p;
  ra.bad = pk.bad.p;
  ra.st = pk.st.p;
  ra.base_words = pk.base_words;
  ra.plane_words = pk.plane_words;
  ra.n = pk.n;
  ra.k = k;
  ra.shards = shards;
  ra.owner = p.owner;
  ra.p1 = (uint32_t)p1;
  ra.h1 = h1.p;
  ra.ctr = ctr;
  mark(ctx, 2, s);
  launch_own_hist(ra, grid, s);
  exclusive_scan_u32(h1.p, (int64_t)nb1 * grid, part.p, s);
  launch_gather_strided(h1.p, (uint64_t)grid, (uint32_t)nb1, b1.p, s);
  HIP_TRY(hipGetLastError());
  std::vector<uint32_t> hb(nb1);
  HIP_TRY(hipMemcpyAsync(hb.data(), b1.p, sizeof(uint32_t) * nb1, hipMemcpyDeviceToHost, s));
  uint64_t c[kCtrCount];
  KH_TRY(read_ctr_at(ctr, s, c));
  if (c[kCtrStatus] & kStatusBadOffsets)
    return fail(KH_EINVAL, "offsets are not non-decreasing from 0 to the base count");
  const uint64_t n_rec = c[kCtrWindows];
  if (n_rec > 0xffffffffull)
    return fail(KH_EOVERFLOW, "%llu windows in one table exceed the 32-bit count",
                (unsigned long long)n_rec);
  t->n_windows = n_rec;
  ctx->last_stats[4] = n_rec;
  ctx->last_stats[10] = k;
  if (n_rec == 0) {
    mark(ctx, 3, s);
    for (int e = 4; e < 12; ++e) mark(ctx, e, s);
    HIP_TRY(hipStreamSynchronize(s));
    accumulate_phases(ctx, 1, 5);
    return KH_OK;
  }
  std::vector<uint64_t> nbk(nb1);
  for (int b = 0; b < nb1; ++b)
    nbk[b] = (b + 1 < nb1 ? (uint64_t)hb[b + 1] : n_rec) - hb[b];

  // ---- level 1 emit
  Buf<uint64_t> rec1(pool), rec2(pool);
  KH_TRY(rec1.alloc(n_rec * R));
  KH_TRY(rec2.alloc(n_rec * R));
  ra.rec = rec1.p;
  launch_own_emit(ra, grid, s);
  HIP_TRY(hipGetLastError());

  // ---- level 2 and the owners; a failed fit splits the owners finer
  const int chunk = own_chunk_records(k);
  const int T = own_slots(k);
  // Testing hook: owners get fewer LDS slots than they are sized for, so
  // that their keys do not fit (the re-split and fallback paths).
  uint32_t slots = (uint32_t)T;
  if (const char* e = std::getenv("KMERHIP_OWNER_SLOTS"))
    slots = (uint32_t)std::max<long long>(16, std::min<long long>(T, std::atoll(e)));
  // Records per owner: with the Bloom screen an owner's table only takes
  // keys seen at least twice, so 2 x slots records always fit (false
  // positives aside); without it, every record may be a new key.  An owner
  // larger than that (a bucket already split by kOwnL2Max bits) may not fit:
  // then every owner is split by two more bits and counted again.
  double target = (p.use_bloom ? 2.0 : 1.0) * T;
  const int p2max = std::max(0, std::min(kOwnL2Max, 2 * (int)k - p1));
  for (int attempt = 0;; ++attempt) {
    // the previous attempt staged its rows over the level-1 records
    if (attempt > 0) launch_own_emit(ra, grid, s);
    std::vector<OwnBucket> bk(nb1);
    uint64_t n_owners = 0, n_chunks = 0, m_size = 0;
    for (int b = 0; b < nb1; ++b) {
      OwnBucket& x = bk[b];
      x.start = hb[b];
      x.n = nbk[b];
      int p2 = 0;
      while (p2 < p2max && (double)x.n / (double)(1u << p2) > target) ++p2;
      x.p2 = (uint32_t)p2;
      x.chunks = (uint32_t)((x.n + chunk - 1) / chunk);
      x.sbbase = (uint32_t)n_owners;
      x.cbase = (uint32_t)n_chunks;
      x.mbase = m_size;
      n_owners += 1ull << p2;
      n_chunks += x.chunks;
      m_size += (uint64_t)x.chunks << p2;
    }
    Buf<OwnBucket> dbk(pool);
    Buf<uint32_t> m(pool), start2(pool), rows_sb(pool), row_off(pool), part2(pool);
    Buf<unsigned long long> stripes(pool);
    Buf<uint16_t> owner_bucket(pool), chunk_bucket(pool);
    Buf<uint8_t> owner_pfx(pool);
    KH_TRY(owner_bucket.alloc(n_owners));
    KH_TRY(owner_pfx.alloc(n_owners));
    KH_TRY(chunk_bucket.alloc(std::max<uint64_t>(n_chunks, 1)));
    KH_TRY(dbk.alloc(nb1));
    KH_TRY(m.alloc(std::max<uint64_t>(m_size, 1)));
    KH_TRY(start2.alloc(n_owners + 1));
    KH_TRY(rows_sb.alloc(n_owners));
    KH_TRY(row_off.alloc(n_owners));
    KH_TRY(part2.alloc(scan_tmp_words((int64_t)n_owners + 1)));
    KH_TRY(stripes.alloc((uint64_t)kOwnStripes * kCtrCount + 1));  // + staging cursor
    HIP_TRY(hipMemcpyAsync(dbk.p, bk.data(), sizeof(OwnBucket) * nb1, hipMemcpyHostToDevice, s));
    OwnPartArgs pa{};
    pa.rec_in = rec1.p;
    pa.rec_out = rec2.p;
    pa.buckets = dbk.p;
    pa.n_buckets = nb1;
    pa.m = m.p;
    pa.start2 = start2.p;
    pa.owner_bucket = owner_bucket.p;
    pa.owner_pfx = owner_pfx.p;
    pa.chunk_bucket = chunk_bucket.p;
    pa.k = k;
    pa.p1 = (uint32_t)p1;
    launch_own_maps(pa, s);
    launch_own_part(pa, (uint32_t)n_chunks, 0, s);
    launch_own_colscan(pa, (uint32_t)n_owners, s);
    exclusive_scan_u32(start2.p, (int64_t)n_owners + 1, part2.p, s);
    launch_own_part(pa, (uint32_t)n_chunks, 1, s);
    HIP_TRY(hipGetLastError());
    mark(ctx, 3, s);

    // ---- the owners.  Their rows are staged in the level-1 record buffer
    // (dead once the level-2 scatter has run; rows are far fewer bytes than
    // records at any useful coverage), blocks taking chunks of it in turn;
    // if it runs out, the pass runs again with staging of exactly the rows,
    // every owner's at its scanned offset.
    const uint32_t blocks =
        (uint32_t)std::min<uint64_t>(n_owners, (uint64_t)ctx->cus * kOwnBlocksPerCU);
    const uint64_t rb = 8ull * W + 4 + 32 + 2;  // key words, count, tallies, codes
    Buf<uint64_t> st_off(pool);
    Buf<uint32_t> st_fixed(pool);
    Buf<uint8_t> st_big(pool);
    uint64_t st_big_bytes = 0;
    KH_TRY(st_off.alloc(n_owners));
    OwnCountArgs ca{};
    // SoA rows in `bytes` at p: keys, counts, tallies, codes (16-byte aligned)
    auto stage_in = [&](uint8_t* p, uint64_t bytes) {
      const uint64_t cap = bytes > 256 ? (bytes - 256) / rb : 0;
      ca.st_cap = cap;
      ca.st_chunk = std::max<uint64_t>(64, cap / (16ull * blocks));
      ca.st_keys = reinterpret_cast<uint64_t*>(p);
      uint8_t* q = p + (cap * 8 * W + 15) / 16 * 16;
      ca.st_counts = reinterpret_cast<uint32_t*>(q);
      q += (cap * 4 + 15) / 16 * 16;
      ca.st_ext = reinterpret_cast<uint32_t*>(q);
      ca.st_codes = q + cap * 32;
    };
    if (p.min_count <= 1 && n_rec * rb > n_rec * R * 8) {
      // every key is a row, and rows take more bytes than records: stage
      // them in a buffer of their own, sized for a row per window plus what
      // the blocks' partly filled staging chunks leave unused
      st_big_bytes = (n_rec + n_rec / 8 + 20ull * blocks * (uint64_t)T) * rb + 512;
      KH_TRY(st_big.alloc(st_big_bytes));
      stage_in(st_big.p, st_big_bytes);
    } else {
      stage_in(reinterpret_cast<uint8_t*>(rec1.p), n_rec * R * 8);
    }
    ca.rec = rec2.p;
    ca.start2 = start2.p;
    ca.owner_bucket = owner_bucket.p;
    ca.n_owners = (uint32_t)n_owners;
    ca.k = k;
    ca.p1 = (uint32_t)p1;
    ca.min_count = p.min_count;
    ca.t_min_ext = p.t_min_ext;
    ca.t_base = p.t_base;
    ca.err_ppm = p.err_ppm;
    ca.use_bloom = p.use_bloom ? 1u : 0u;
    ca.slots = slots;
    ca.st_off = st_off.p;
    ca.st_cursor = stripes.p + (size_t)kOwnStripes * kCtrCount;
    ca.rows_sb = rows_sb.p;
    ca.row_off = row_off.p;
    ca.ctr = stripes.p;
    const bool dbg = std::getenv("KMERHIP_OWNER_DEBUG") != nullptr;
    Buf<unsigned long long> prof(pool);
    if (dbg) {
      KH_TRY(prof.alloc(8));
      ca.prof = prof.p;
    }
    mark(ctx, 4, s);
    for (int pass = 0;; ++pass) {
      launch_fill_u64(reinterpret_cast<uint64_t*>(stripes.p),
                      (uint64_t)kOwnStripes * kCtrCount + 1, 0ull, s);
      if (dbg) launch_fill_u64(reinterpret_cast<uint64_t*>(prof.p), 8, 0ull, s);
      launch_own_count(ca, blocks, s);
      HIP_TRY(hipGetLastError());
      std::vector<uint64_t> hs((size_t)kOwnStripes * kCtrCount);
      HIP_TRY(hipMemcpyAsync(hs.data(), stripes.p, hs.size() * 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      std::memset(c, 0, sizeof c);
      for (int q = 0; q < kOwnStripes; ++q) {
        const uint64_t* x = &hs[(size_t)q * kCtrCount];
        c[kCtrStatus] |= x[kCtrStatus];
        c[kCtrWindows] = std::max(c[kCtrWindows], x[kCtrWindows]);
        for (int e : {kCtrL1New, kCtrL2New, kCtrRows, kCtrClaimed, kCtrHeavy, kCtrPassed})
          c[e] += x[e];
      }
      if (dbg) {
        uint64_t pc[8];
        HIP_TRY(hipMemcpy(pc, prof.p, sizeof pc, hipMemcpyDeviceToHost));
        std::fprintf(stderr, "owner k=%u phase clocks per owner:", k);
        for (int e = 0; e < 8; ++e) std::fprintf(stderr, " %.0f", (double)pc[e] / n_owners);
        std::fprintf(stderr, "\n");
      }
      if (pass > 0 || (c[kCtrStatus] & kStatusProbeLimit) || !(c[kCtrStatus] & kStatusStaging))
        break;
      // every owner wrote its row count to row_off: scan a copy into the
      // owners' staging offsets
      if (dbg)
        std::fprintf(stderr, "owner k=%u staging of %llu rows ran out: %llu rows\n", k,
                     (unsigned long long)ca.st_cap, (unsigned long long)c[kCtrRows]);
      KH_TRY(st_fixed.alloc(n_owners));
      HIP_TRY(hipMemcpyAsync(st_fixed.p, row_off.p, n_owners * 4, hipMemcpyDeviceToDevice, s));
      exclusive_scan_u32(st_fixed.p, (int64_t)n_owners, part2.p, s);
      st_big_bytes = c[kCtrRows] * rb + 512;
      KH_TRY(st_big.alloc(st_big_bytes));
      stage_in(st_big.p, st_big_bytes);
      ca.st_fixed = st_fixed.p;
    }
    mark(ctx, 5, s);
    mark(ctx, 6, s);
    exclusive_scan_u32(row_off.p, (int64_t)n_owners, part2.p, s);
    mark(ctx, 7, s);
    mark(ctx, 8, s);
    mark(ctx, 9, s);
    ctx->last_stats[9] += c[kCtrHeavy];
    ctx->last_stats[11] = c[kCtrWindows];
    if (std::getenv("KMERHIP_OWNER_DEBUG"))
      std::fprintf(stderr, "owner k=%u attempt %d: owners %llu chunks %llu matrix %llu, "
                   "%llu did not fit, largest %llu keys (slots %u), target %.0f records\n",
                   k, attempt, (unsigned long long)n_owners, (unsigned long long)n_chunks,
                   (unsigned long long)m_size, (unsigned long long)c[kCtrHeavy],
                   (unsigned long long)c[kCtrWindows], slots, target);
    if (c[kCtrStatus] & kStatusProbeLimit) {
      if (attempt >= 2) {
        *unfit = true;
        return KH_OK;
      }
      target /= 4.0;  // two more key bits per owner
      continue;
    }
    const int64_t rows = (int64_t)c[kCtrRows];
    if (t->dst_cap >= 0 && rows > t->dst_cap) {
      t->n_rows = rows;
      return fail(KH_EOVERFLOW, "%lld rows do not fit the %lld rows of the output buffers",
                  (long long)rows, (long long)t->dst_cap);
    }
    ctx->last_stats[0] = n_owners * slots;
    ctx->last_stats[1] = c[kCtrClaimed];
    ctx->last_stats[2] = c[kCtrL1New];
    ctx->last_stats[3] = c[kCtrL2New];
    ctx->last_stats[5] = (uint64_t)rows;
    ctx->last_stats[6] = (uint64_t)attempt;
    ctx->last_stats[7] = 2 * n_rec * R * 8 + st_big_bytes;
    ctx->last_stats[8] = c[kCtrPassed];

    Buf<uint32_t> counts(pool), ext(pool);
    Buf<uint8_t> codes(pool);
    Buf<uint64_t> keys(pool);
    const bool to_caller = t->dst_cap >= 0;
    if (!to_caller) {
      KH_TRY(keys.alloc((uint64_t)rows * W));
      KH_TRY(counts.alloc((uint64_t)rows));
      KH_TRY(ext.alloc((uint64_t)rows * 8));
      KH_TRY(codes.alloc((uint64_t)rows * 2));
    }
    OwnCopyArgs oa{};
    oa.owner_pfx = owner_pfx.p;
    oa.k = k;
    oa.st_keys = ca.st_keys;
    oa.st_counts = ca.st_counts;
    oa.st_ext = ca.st_ext;
    oa.st_codes = ca.st_codes;
    oa.rows_sb = rows_sb.p;
    oa.row_off = row_off.p;
    oa.st_off = st_off.p;
    oa.W = (uint32_t)W;
    oa.keys = to_caller ? t->dst_keys : keys.p;
    oa.counts = to_caller ? t->dst_counts : counts.p;
    oa.ext = to_caller ? t->dst_ext : ext.p;
    oa.codes = to_caller ? t->dst_codes : codes.p;
    mark(ctx, 10, s);
    if (rows > 0) launch_own_copy(oa, (uint32_t)n_owners, s);
    HIP_TRY(hipGetLastError());
    mark(ctx, 11, s);
    HIP_TRY(hipStreamSynchronize(s));
    t->n_rows = rows;
    if (!to_caller) {
      t->keys = keys.release();
      t->counts = counts.release();
      t->ext = ext.release();
      t->codes = codes.release();
    }
    accumulate_phases(ctx, 1, 5);
    if (ctx->cur_k < kMaxK)
      std::memcpy(ctx->k_stats[ctx->cur_k], ctx->last_stats, sizeof ctx->last_stats);
    return KH_OK;
  }
}

// Count one k over packed reads into the table object t.
// ctx->ctr[kCtrStatus] carries the pack stage's status (bad offsets are
// reported here).
static int count_packed_into(kh_ctx* ctx, Packed& pk, const kh_params& p,
                             hipStream_t s, kh_table* t) {
  const uint32_t k = p.k;
  const int ws = table_chunks(k);
  const SlotLayout lay = slot_layout(ws);
  std::memset(ctx->last_stats, 0, sizeof ctx->last_stats);
  if (pk.n == 0) {
    HIP_TRY(hipStreamSynchronize(s));
    return KH_OK;
  }
  Pool* pool = &ctx->pool;
  if (owned_applies(ctx)) {
    // The owner path holds two record buffers (16 x own_record_words(k)
    // bytes per window); where the budget refuses them, or some owner's keys
    // never fit, the single-table path counts this k.
    bool unfit = false;
    const int rc = count_owned(ctx, pk, p, s, t, &unfit);
    if (rc != KH_OK && rc != KH_ENOMEM) return rc;
    if (rc == KH_OK && !unfit) return KH_OK;
    if (rc == KH_ENOMEM) HIP_TRY(hipStreamSynchronize(s));
    std::memset(ctx->last_stats, 0, sizeof ctx->last_stats);
  }
  const double lf = p.load_factor > 0.0f ? (double)p.load_factor : ctx->tune.load_factor;

  // reset the per-count counters; the pack stage's status bit stays
  uint64_t c[kCtrCount];
  launch_reset_ctr(ctx->ctr, kStatusBadOffsets, s);
  bool timed_bloom = false;

  WindowArgs wa{};
  wa.bases = pk.bases.p;
  wa.hq = pk.hq.p;
  wa.bad = pk.bad.p;
  wa.st = pk.st.p;
  wa.base_words = pk.base_words;
  wa.plane_words = pk.plane_words;
  wa.n = pk.n;
  wa.k = k;
  wa.ctr = ctx->ctr;
  wa.tiles_per_block = (int)ctx->tune.tiles_per_block;
  wa.lanes = (int)ctx->tune.count_lanes;
  wa.aggregate = (int)ctx->tune.aggregate;
  const uint32_t shards = p.owner_shards > 1 ? p.owner_shards : 1;
  wa.shards = shards;
  wa.owner = p.owner;

  // ---- Bloom pass A: which keys are seen at least twice
  Buf<uint64_t> bloom(pool), seen(pool);
  uint64_t est;
  uint64_t n_windows = 0;
  if (p.use_bloom) {
    // one 64-bit word (32 bits per level) per `bits` bits of each level per
    // base position
    const uint64_t bits = p.bloom_bits ? p.bloom_bits : ctx->tune.bloom_bits;
    uint64_t blocks = ((uint64_t)pk.n * bits + 32 * shards - 1) / (32 * shards);
    blocks = std::max<uint64_t>(blocks, 64);
    KH_TRY(bloom.alloc(blocks));
    launch_fill_u64(bloom.p, blocks, 0ull, s);
    wa.bloom = bloom.p;
    wa.bloom_blocks = blocks;
    // sighting bits of every window position pass A visits (it writes all)
    KH_TRY(seen.alloc((uint64_t)((pk.n + kTile - 1) / kTile) * (kTile / 64)));
    wa.seen = seen.p;
    mark(ctx, 2, s);
    WindowArgs wb = wa;
    wb.lanes = (int)ctx->tune.bloom_lanes;
    if (pk.packed == pk.n) {
      launch_windows(wb, 1, s);
    } else {
      // streamed host reads: pass A over the tiles already packed while the
      // next chunk copies on the side stream (as in the batched call)
      const int64_t n_tiles = (pk.n + kTile - 1) / kTile;
      const int64_t chunk = stream_chunk_bases();
      int64_t t_done = 0;
      while (pk.packed < pk.n) {
        const int64_t p1 = std::min(pk.n, pk.packed + chunk);
        KH_TRY(stream_chunk(ctx, pk, pk.packed, p1, s, ctx->side));
        const int64_t ready =
            p1 == pk.n ? n_tiles
                       : std::max<int64_t>(0, (p1 - (kSpan - kHalo) - 64) / kTile);
        if (ready > t_done) {
          wb.t_begin = t_done;
          wb.t_end = ready;
          launch_windows(wb, 1, s);
        }
        t_done = std::max(t_done, ready);
      }
    }
    HIP_TRY(hipGetLastError());
    mark(ctx, 3, s);
    timed_bloom = true;
    KH_TRY(read_ctr(ctx, s, c));
    if (c[kCtrStatus] & kStatusBadOffsets)
      return fail(KH_EINVAL, "offsets are not non-decreasing from 0 to the base count");
    n_windows = c[kCtrWindows];
    const double l1 = (double)c[kCtrL1New], l2 = (double)c[kCtrL2New];
    // keys inserted in pass B: level-2 patterns completed, plus singletons
    // whose level-2 pattern is complete by chance
    const double dens = 1.0 - std::exp(-4.0 * l2 / (32.0 * (double)blocks));
    const double fp = std::pow(dens, 4.0);
    est = (uint64_t)(l2 * 1.05 + fp * std::max(0.0, l1 - l2) * 2.0) + 1024;
    ctx->last_stats[2] = c[kCtrL1New];
    ctx->last_stats[3] = c[kCtrL2New];
  } else {
    est = (uint64_t)pk.n / shards + 1024;
  }

  // ---- count pass B (grow and retry if a probe runs out)
  uint64_t cap = (uint64_t)std::ceil((double)est / lf);
  cap = std::max<uint64_t>(cap, 1024);
  // Test hook: start from a given (too small) capacity to exercise the
  // rebuild path.  The rebuild doubles the table until every key fits.
  if (const char* force = std::getenv("KMERHIP_FORCE_CAPACITY"))
    cap = std::max<uint64_t>(64, std::strtoull(force, nullptr, 10));
  // A fixed scratch range (arena mode) bounds the table: besides its slots
  // it must hold the classify output (12 B per slot), the sort's second
  // buffers (at most 12 B per slot) and the heavy-hitter list.
  uint64_t arena_cap = 0;
  if (pool->arena) {
    const uint64_t reserve = (uint64_t)kHeavyMax * 4 + (2ull << 20);
    const uint64_t room = pool->arena_free() > reserve ? pool->arena_free() - reserve : 0;
    arena_cap = room / (lay.stride + 26);
    if (arena_cap < 64)
      return fail(KH_ENOMEM, "the no-allocation scratch has no room left for a table "
                             "(%llu bytes free)", (unsigned long long)pool->arena_free());
    cap = std::min(cap, arena_cap);
  }
  Buf<uint8_t> table(pool);
  int retries = 0;
  for (;;) {
    if (cap >= (1ull << 32))
      return fail(KH_ENOMEM, "table capacity %llu exceeds 2^32 slots",
                  (unsigned long long)cap);
    KH_TRY(table.alloc(cap * lay.stride));
    launch_fill_u64(reinterpret_cast<uint64_t*>(table.p), cap * lay.stride / 8,
                    0ull, s);
    wa.table = table.p;
    wa.capacity = cap;
    wa.max_probe = (uint32_t)std::min<uint64_t>(cap, 1u << 14);
    // a capped table (arena mode) may truly fill up: shorter probe chains
    // keep every window's search short when it does
    if (pool->arena) wa.max_probe = std::min<uint32_t>(wa.max_probe, 1024);
    wa.count_windows = p.use_bloom ? 0 : 1;
    mark(ctx, 4, s);
    launch_windows(wa, p.use_bloom ? 2 : 0, s);
    HIP_TRY(hipGetLastError());
    mark(ctx, 5, s);
    KH_TRY(read_ctr(ctx, s, c));
    if (c[kCtrStatus] & kStatusBadOffsets)
      return fail(KH_EINVAL, "offsets are not non-decreasing from 0 to the base count");
    if (!(c[kCtrStatus] & kStatusProbeLimit)) break;
    // the table was too small for the keys it received: start pass B over
    ++retries;
    if (pool->arena) {
      if (cap >= arena_cap)
        return fail(KH_ENOMEM, "the k-mers do not fit the largest table the no-allocation "
                               "scratch holds (%llu slots)", (unsigned long long)arena_cap);
      cap = std::min(2 * cap, arena_cap);
    } else {
      cap *= 2;
    }
    launch_reset_ctr(ctx->ctr, 0, s);
  }
  if (!p.use_bloom) n_windows = c[kCtrWindows];
  if (n_windows > 0xffffffffull)
    return fail(KH_EOVERFLOW, "%llu windows in one table exceed the 32-bit count",
                (unsigned long long)n_windows);
  ctx->last_stats[0] = cap;
  ctx->last_stats[1] = c[kCtrClaimed];
  ctx->last_stats[4] = n_windows;
  ctx->last_stats[6] = (uint64_t)retries;
  ctx->last_stats[7] = cap * lay.stride;
  ctx->last_stats[8] = c[kCtrPassed];

  RecountFn recount = [&](HeavyEntry* heavy, uint32_t* index, uint32_t mask) -> int {
    WindowArgs wh = wa;
    wh.heavy = heavy;
    wh.heavy_index = index;
    wh.heavy_mask = mask;
    launch_windows(wh, 3, s);
    return KH_OK;
  };
  t->n_windows = n_windows;
  KH_TRY(finish_rows(ctx, ctx->ctr, table.p, cap, p, recount, s, t));
  accumulate_phases(ctx, timed_bloom ? 1 : 2, 5);
  if (ctx->cur_k < kMaxK)
    std::memcpy(ctx->k_stats[ctx->cur_k], ctx->last_stats, sizeof ctx->last_stats);
  return KH_OK;
}

// Count one k over packed reads into a new table.
static int count_packed(kh_ctx* ctx, Packed& pk, const kh_params& p,
                        hipStream_t s, kh_table** out) {
  kh_table* t = nullptr;
  KH_TRY(make_table(ctx, p.k, &t));
  const int rc = count_packed_into(ctx, pk, p, s, t);
  if (rc != KH_OK) {
    kh_table_free(t);
    return rc;
  }
  *out = t;
  return KH_OK;
}

int kh::count_into(kh_ctx* ctx, const kh_reads* reads, const kh_params& p, hipStream_t s,
                   kh_table* t) {
  Packed pk(&ctx->pool);
  KH_TRY(pack_reads(ctx, reads, p, s, pk, false));
  return count_packed_into(ctx, pk, p, s, t);
}

// Batched multi-k: fused Bloom launches (one per key width; for streamed
// host reads, one set per uploaded chunk over the tiles it completes), one
// planning synchronisation for all k, the counting passes of every k
// captured in one hipGraph, and each k's tail (classify, heavy recount,
// sort, gather) on the side stream as soon as its counting pass has
// finished, overlapping the counting passes of the later k.  Tables are
// bit-identical to kh_count.
static int count_multi_batched(kh_ctx* ctx, Packed& pk, const kh_params& base,
                               const uint32_t* ks, int nk, hipStream_t s,
                               kh_table** outs) {
  Pool* pool = &ctx->pool;
  hipStream_t s2 = ctx->side;
  const double lf = base.load_factor > 0.0f ? (double)base.load_factor : ctx->tune.load_factor;
  kh_table* tabs[kMaxK] = {};
  struct Cleanup {
    kh_table** t;
    int n;
    bool keep = false;
    ~Cleanup() {
      if (!keep)
        for (int i = 0; i < n; ++i) kh_table_free(t[i]);
    }
  } cleanup{tabs, nk};
  for (int i = 0; i < nk; ++i) KH_TRY(make_table(ctx, ks[i], &tabs[i]));
  if (pk.n == 0) {
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < nk; ++i) outs[i] = tabs[i];
    cleanup.keep = true;
    return KH_OK;
  }
  unsigned long long* kc = ctx->kctr;
  launch_fill_u64(reinterpret_cast<uint64_t*>(kc), (uint64_t)kMaxK * kCtrCount, 0ull, s);
  const uint32_t shards = base.owner_shards > 1 ? base.owner_shards : 1;

  WindowArgs wa[kMaxK];
  for (int i = 0; i < nk; ++i) {
    wa[i] = WindowArgs{};
    wa[i].bases = pk.bases.p;
    wa[i].hq = pk.hq.p;
    wa[i].bad = pk.bad.p;
    wa[i].st = pk.st.p;
    wa[i].base_words = pk.base_words;
    wa[i].plane_words = pk.plane_words;
    wa[i].n = pk.n;
    wa[i].k = ks[i];
    wa[i].ctr = kc + (size_t)i * kCtrCount;
    wa[i].tiles_per_block = (int)ctx->tune.tiles_per_block;
    wa[i].lanes = (int)ctx->tune.count_lanes;
    wa[i].aggregate = (int)ctx->tune.aggregate;
    wa[i].shards = shards;
    wa[i].owner = base.owner;
  }
  // ---- Bloom pass A for every k: one fused launch per key width
  Buf<uint64_t> bloom[kMaxK], seen[kMaxK];
  uint64_t est[kMaxK];
  uint64_t c[kCtrCount];
  std::vector<uint64_t> hc((size_t)kMaxK * kCtrCount);
  bool timed_bloom = false;
  if (base.use_bloom) {
    const uint64_t bits = base.bloom_bits ? base.bloom_bits : ctx->tune.bloom_bits;
    std::vector<int> order;  // k indices grouped by key width
    for (int w = 1; w <= 4; ++w)
      for (int i = 0; i < nk; ++i)
        if ((int)(ks[i] + 31) / 32 == w) order.push_back(i);
    std::vector<BloomSlot> hs(nk);
    for (int j = 0; j < nk; ++j) {
      const int i = order[j];
      bloom[i].pool = pool;
      seen[i].pool = pool;
      const uint64_t blocks =
          std::max<uint64_t>(((uint64_t)pk.n * bits + 32 * shards - 1) / (32 * shards), 64);
      KH_TRY(bloom[i].alloc(blocks));
      launch_fill_u64(bloom[i].p, blocks, 0ull, s);
      KH_TRY(seen[i].alloc((uint64_t)((pk.n + kTile - 1) / kTile) * (kTile / 64)));
      wa[i].bloom = bloom[i].p;
      wa[i].bloom_blocks = blocks;
      wa[i].seen = seen[i].p;
      hs[j] = BloomSlot{ks[i], 0, bloom[i].p, blocks, wa[i].ctr, seen[i].p};
    }
    Buf<BloomSlot> ds(pool);
    KH_TRY(ds.alloc(nk));
    HIP_TRY(hipMemcpyAsync(ds.p, hs.data(), nk * sizeof(BloomSlot), hipMemcpyHostToDevice, s));
    mark(ctx, 2, s);
    // Bloom pass A over tiles [t0, t1) for every k: one launch per key width
    auto bloom_tiles = [&](int64_t t0, int64_t t1) -> int {
    for (int j = 0; j < nk;) {
      const int w = (int)(ks[order[j]] + 31) / 32;
      int e = j;
      while (e < nk && e - j < kBloomFuse && (int)(ks[order[e]] + 31) / 32 == w) ++e;
      MultiBloomArgs ma{};
      ma.t_begin = t0;
      ma.t_end = t1;
      ma.bases = pk.bases.p;
      ma.hq = pk.hq.p;
      ma.bad = pk.bad.p;
      ma.st = pk.st.p;
      ma.base_words = pk.base_words;
      ma.plane_words = pk.plane_words;
      ma.n = pk.n;
      ma.nk = e - j;
      ma.k0 = ks[order[j]];
      ma.slots = ds.p + j;
      ma.lanes = (int)ctx->tune.bloom_lanes;
      ma.tiles_per_block = (int)ctx->tune.tiles_per_block;
      ma.shards = shards;
      ma.owner = base.owner;
      launch_bloom_multi(ma, s);
      HIP_TRY(hipGetLastError());
      j = e;
    }
    return KH_OK;
    };
    const int64_t n_tiles = (pk.n + kTile - 1) / kTile;
    if (pk.packed == pk.n) {
      KH_TRY(bloom_tiles(0, n_tiles));
    } else {
      // streamed host reads: chunk c's copy runs on the side stream while
      // the Bloom launches over the tiles already packed run on s.  A tile
      // is ready once every position it stages (up to kSpan - kHalo past
      // its first window, plus a word of rounding) is packed.
      const int64_t chunk = stream_chunk_bases();
      int64_t t_done = 0;
      while (pk.packed < pk.n) {
        const int64_t p1 = std::min(pk.n, pk.packed + chunk);
        KH_TRY(stream_chunk(ctx, pk, pk.packed, p1, s, s2));
        const int64_t ready =
            p1 == pk.n ? n_tiles
                       : std::max<int64_t>(0, (p1 - (kSpan - kHalo) - 64) / kTile);
        if (ready > t_done) KH_TRY(bloom_tiles(t_done, ready));
        t_done = std::max(t_done, ready);
      }
    }
    mark(ctx, 3, s);
    timed_bloom = true;
    HIP_TRY(hipMemcpyAsync(hc.data(), kc, hc.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < nk; ++i) {
      const uint64_t* ci = &hc[(size_t)i * kCtrCount];
      const double l1 = (double)ci[kCtrL1New], l2 = (double)ci[kCtrL2New];
      const double dens = 1.0 - std::exp(-4.0 * l2 / (32.0 * (double)wa[i].bloom_blocks));
      const double fp = std::pow(dens, 4.0);
      est[i] = (uint64_t)(l2 * 1.05 + fp * std::max(0.0, l1 - l2) * 2.0) + 1024;
    }
  } else {
    for (int i = 0; i < nk; ++i) est[i] = (uint64_t)pk.n / shards + 1024;
  }
  KH_TRY(read_ctr(ctx, s, c));  // the pack stage's status
  if (c[kCtrStatus] & kStatusBadOffsets)
    return fail(KH_EINVAL, "offsets are not non-decreasing from 0 to the base count");

  // ---- tables for every k, then the counting passes as one graph
  Buf<uint8_t> table[kMaxK];
  uint64_t cap[kMaxK];
  const char* force = std::getenv("KMERHIP_FORCE_CAPACITY");
  for (int i = 0; i < nk; ++i) {
    const SlotLayout lay = slot_layout(table_chunks(ks[i]));
    cap[i] = std::max<uint64_t>((uint64_t)std::ceil((double)est[i] / lf), 1024);
    if (force) cap[i] = std::max<uint64_t>(64, std::strtoull(force, nullptr, 10));
    if (cap[i] >= (1ull << 32))
      return fail(KH_ENOMEM, "table capacity %llu exceeds 2^32 slots",
                  (unsigned long long)cap[i]);
    table[i].pool = pool;
    KH_TRY(table[i].alloc(cap[i] * lay.stride));
    wa[i].table = table[i].p;
    wa[i].capacity = cap[i];
    wa[i].max_probe = (uint32_t)std::min<uint64_t>(cap[i], 1u << 14);
    wa[i].count_windows = base.use_bloom ? 0 : 1;
  }
  const int mode = base.use_bloom ? 2 : 0;
  // ---- the counting passes of every k as one graph.  They are captured on
  // the context's own stream (the caller's may be the null stream, which
  // cannot be captured; capture runs nothing) as a chain fill_0, pass_0,
  // fill_1, pass_1, ...  An event recorded on a capturing stream does not
  // become a node the outside can wait on, so each pass then gets
  // event-record nodes added to the captured graph, one between its fill and
  // itself and one between itself and the next fill, keeping the graph one
  // chain (a leaf event node may be recorded only when the whole graph
  // ends); the side stream's tails wait on the pass-end events.  The graph is launched on the caller's stream and kept for the
  // next call (updated in place when the topology matches).  Any failure:
  // the same launches, eagerly.  Testing hook: KMERHIP_NO_GRAPH=1.
  auto tail_node = [](hipStream_t q, hipGraphNode_t* out) -> bool {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    const hipGraphNode_t* deps = nullptr;
    size_t nd = 0;
    if (hipStreamGetCaptureInfo_v2(q, &st, nullptr, nullptr, &deps, &nd) != hipSuccess ||
        st != hipStreamCaptureStatusActive || nd != 1 || !deps)
      return false;
    *out = deps[0];
    return true;
  };
  const char* no_graph = std::getenv("KMERHIP_NO_GRAPH");
  hipStream_t cs = ctx->capture;
  bool graphed = false;
  if (!(no_graph && no_graph[0] == '1') &&
      hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    hipGraphNode_t fill_n[kMaxK] = {}, pass_n[kMaxK] = {};
    bool ok = true;
    for (int i = 0; i < nk; ++i) {
      const SlotLayout lay = slot_layout(table_chunks(ks[i]));
      launch_fill_u64(reinterpret_cast<uint64_t*>(table[i].p), cap[i] * lay.stride / 8,
                      0ull, cs);
      ok = ok && tail_node(cs, &fill_n[i]);
      launch_windows(wa[i], mode, cs);
      ok = ok && tail_node(cs, &pass_n[i]);
    }
    hipGraph_t graph = nullptr;
    ok = hipStreamEndCapture(cs, &graph) == hipSuccess && graph && ok;
    for (int i = 0; ok && i < nk; ++i) {
      hipGraphNode_t e0 = nullptr, e1 = nullptr;
      ok = hipGraphRemoveDependencies(graph, &fill_n[i], &pass_n[i], 1) == hipSuccess &&
           hipGraphAddEventRecordNode(&e0, graph, &fill_n[i], 1, ctx->kev[i][0]) == hipSuccess &&
           hipGraphAddDependencies(graph, &e0, &pass_n[i], 1) == hipSuccess &&
           hipGraphAddEventRecordNode(&e1, graph, &pass_n[i], 1, ctx->kev[i][1]) == hipSuccess;
      if (ok && i + 1 < nk)  // pass_i -> e1 -> fill_i+1 instead of pass_i -> fill_i+1
        ok = hipGraphRemoveDependencies(graph, &pass_n[i], &fill_n[i + 1], 1) == hipSuccess &&
             hipGraphAddDependencies(graph, &e1, &fill_n[i + 1], 1) == hipSuccess;
    }
    if (ok) {
      bool ready = false;
      if (ctx->graph_exec) {  // same topology as last time: update in place
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        ready = hipGraphExecUpdate(ctx->graph_exec, graph, &err_node, &res) == hipSuccess &&
                res == hipGraphExecUpdateSuccess;
        if (!ready) {
          (void)hipGetLastError();
          (void)hipGraphExecDestroy(ctx->graph_exec);
          ctx->graph_exec = nullptr;
        }
      }
      if (!ready)
        ready = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0) == hipSuccess;
      ok = ready && hipGraphLaunch(ctx->graph_exec, s) == hipSuccess;
    }
    if (graph) (void)hipGraphDestroy(graph);
    graphed = ok;
  }
  if (!graphed) {  // the same launches, eagerly
    (void)hipGetLastError();
    for (int i = 0; i < nk; ++i) {
      const SlotLayout lay = slot_layout(table_chunks(ks[i]));
      launch_fill_u64(reinterpret_cast<uint64_t*>(table[i].p), cap[i] * lay.stride / 8,
                      0ull, s);
      HIP_TRY(hipEventRecord(ctx->kev[i][0], s));
      launch_windows(wa[i], mode, s);
      HIP_TRY(hipEventRecord(ctx->kev[i][1], s));
    }
  }
  ctx->last_graphed = graphed ? 1 : 0;
  HIP_TRY(hipGetLastError());

  // ---- per-k tails on the side stream
  for (int i = 0; i < nk; ++i) {
    kh_params p = base;
    p.k = ks[i];
    ctx->cur_k = i;
    const SlotLayout lay = slot_layout(table_chunks(ks[i]));
    unsigned long long* ci = kc + (size_t)i * kCtrCount;
    // the tail of k_i starts when its pass ends, or when the last pass ends
    HIP_TRY(hipStreamWaitEvent(s2, ctx->kev[ctx->tune.tails_overlap ? i : nk - 1][1], 0));
    KH_TRY(read_ctr_at(ci, s2, c));
    float count_ms = 0.0f;
    if (hipEventElapsedTime(&count_ms, ctx->kev[i][0], ctx->kev[i][1]) != hipSuccess) {
      (void)hipGetLastError();
      count_ms = 0.0f;
    }
    int retries = 0;
    while (c[kCtrStatus] & kStatusProbeLimit) {  // rare: rebuild this k's table
      HIP_TRY(hipStreamSynchronize(s));
      ++retries;
      cap[i] *= 2;
      if (cap[i] >= (1ull << 32)) return fail(KH_ENOMEM, "table capacity exceeds 2^32 slots");
      KH_TRY(table[i].alloc(cap[i] * lay.stride));
      launch_fill_u64(reinterpret_cast<uint64_t*>(table[i].p), cap[i] * lay.stride / 8, 0ull, s2);
      launch_reset_ctr(ci, 0, s2);
      wa[i].table = table[i].p;
      wa[i].capacity = cap[i];
      wa[i].max_probe = (uint32_t)std::min<uint64_t>(cap[i], 1u << 14);
      launch_windows(wa[i], mode, s2);
      HIP_TRY(hipGetLastError());
      KH_TRY(read_ctr_at(ci, s2, c));
    }
    const uint64_t n_windows =
        base.use_bloom ? hc[(size_t)i * kCtrCount + kCtrWindows] : c[kCtrWindows];
    if (n_windows > 0xffffffffull)
      return fail(KH_EOVERFLOW, "%llu windows in one table exceed the 32-bit count",
                  (unsigned long long)n_windows);
    std::memset(ctx->last_stats, 0, sizeof ctx->last_stats);
    ctx->last_stats[0] = cap[i];
    ctx->last_stats[1] = c[kCtrClaimed];
    if (base.use_bloom) {
      ctx->last_stats[2] = hc[(size_t)i * kCtrCount + kCtrL1New];
      ctx->last_stats[3] = hc[(size_t)i * kCtrCount + kCtrL2New];
    }
    ctx->last_stats[4] = n_windows;
    ctx->last_stats[6] = (uint64_t)retries;
    ctx->last_stats[7] = cap[i] * lay.stride;
    ctx->last_stats[8] = c[kCtrPassed];
    RecountFn recount = [&](HeavyEntry* heavy, uint32_t* index, uint32_t mask) -> int {
      WindowArgs wh = wa[i];
      wh.heavy = heavy;
      wh.heavy_index = index;
      wh.heavy_mask = mask;
      launch_windows(wh, 3, s2);
      return KH_OK;
    };
    tabs[i]->n_windows = n_windows;
    KH_TRY(finish_rows(ctx, ci, table[i].p, cap[i], p, recount, s2, tabs[i]));
    accumulate_phases(ctx, 3, 5);
    ctx->last_ms[2] += count_ms;
    ctx->k_ms[i][2] += count_ms;
    std::memcpy(ctx->k_stats[i], ctx->last_stats, sizeof ctx->last_stats);
    table[i].reset();
    bloom[i].reset();
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (timed_bloom && ctx->timing) {  // fused Bloom launches: booked on the first k
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]) == hipSuccess) {
      ctx->last_ms[1] += ms;
      ctx->k_ms[0][1] += ms;
    } else {
      (void)hipGetLastError();
    }
  }
  for (int i = 0; i < nk; ++i) outs[i] = tabs[i];
  cleanup.keep = true;
  return KH_OK;
}

static void start_timing(kh_ctx* ctx) {
  for (float& v : ctx->last_ms) v = 0.0f;
  std::memset(ctx->k_ms, 0, sizeof ctx->k_ms);
  std::memset(ctx->k_stats, 0, sizeof ctx->k_stats);
  ctx->cur_k = 0;
}

namespace kh {
DeviceCache& device_cache(int device) {
  static DeviceCache caches[kMaxDevices];
  return caches[device];
}
}  // namespace kh

// ----------------------------------------------------------------- API ----

extern "C" int kh_create(kh_ctx** out, int device, uint64_t hbm_budget_bytes,
                         kh_alloc_fn alloc_fn, kh_free_fn free_fn, void* user) {
  if (!out) return fail(KH_EINVAL, "out is NULL");
  *out = nullptr;
  if (!alloc_fn != !free_fn) return fail(KH_EINVAL, "give both alloc_fn and free_fn, or neither");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(KH_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= n || device >= kMaxDevices)
    return fail(KH_EINVAL, "device %d out of range", device);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(KH_EDEVICE, "device %d is %s; this library is built for gfx950",
                device, prop.gcnArchName);
  HIP_TRY(hipSetDevice(device));
  kh_ctx* ctx = new (std::nothrow) kh_ctx();
  if (!ctx) return fail(KH_ENOMEM, "host allocation failed");
  ctx->device = device;
  ctx->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  ctx->pool.device = device;
  ctx->pool.budget = hbm_budget_bytes;
  ctx->pool.alloc_fn = alloc_fn;
  ctx->pool.free_fn = free_fn;
  ctx->pool.user = user;
  kh_default_tuning(&ctx->tune);
  // counters live in the pool like everything else (freed with it)
  void* c = nullptr;
  void* kc = nullptr;
  if (ctx->pool.get(&c, sizeof(uint64_t) * kCtrCount) != KH_OK ||
      ctx->pool.get(&kc, sizeof(uint64_t) * kCtrCount * kMaxK) != KH_OK) {
    ctx->pool.release_all();
    delete ctx;
    return fail(KH_ENOMEM, "counter allocation failed");
  }
  ctx->ctr = static_cast<unsigned long long*>(c);
  ctx->kctr = static_cast<unsigned long long*>(kc);
  if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess) {
    ctx->pool.release_all();
    delete ctx;
    return fail(KH_EDEVICE, "stream creation failed");
  }
  if (hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking) != hipSuccess) {
    (void)hipStreamDestroy(ctx->side);
    ctx->pool.release_all();
    delete ctx;
    return fail(KH_EDEVICE, "stream creation failed");
  }
  if (hipEventCreateWithFlags(&ctx->copy_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(ctx->capture);
    (void)hipStreamDestroy(ctx->side);
    ctx->pool.release_all();
    delete ctx;
    return fail(KH_EDEVICE, "event creation failed");
  }
  for (int i = 0; i < kTimeEvents; ++i) (void)hipEventCreate(&ctx->ev[i]);
  for (int i = 0; i < kMaxK; ++i)
    for (int j = 0; j < 2; ++j) (void)hipEventCreate(&ctx->kev[i][j]);
  *out = ctx;
  return KH_OK;
}

extern "C" int kh_destroy(kh_ctx* ctx) {
  if (!ctx) return fail(KH_EINVAL, "ctx is NULL");
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->pool.release_all();
  for (kh_table* t : ctx->live) {  // rows are gone with the pool
    t->ctx = nullptr;
    t->n_rows = 0;
    t->keys = nullptr;
    t->counts = nullptr;
    t->ext = nullptr;
    t->codes = nullptr;
  }
  ctx->live.clear();
  kh_orphan_contigs(ctx);
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  (void)hipStreamDestroy(ctx->side);
  (void)hipStreamDestroy(ctx->capture);
  (void)hipEventDestroy(ctx->copy_ev);
  for (int i = 0; i < kTimeEvents; ++i) (void)hipEventDestroy(ctx->ev[i]);
  for (int i = 0; i < kMaxK; ++i)
    for (int j = 0; j < 2; ++j) (void)hipEventDestroy(ctx->kev[i][j]);
  delete ctx;
  return KH_OK;
}

extern "C" int kh_trim(kh_ctx* ctx) {
  if (!ctx) return fail(KH_EINVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipDeviceSynchronize());
  ctx->pool.drop_cached();
  return KH_OK;
}

extern "C" int kh_release_cached(int device) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(KH_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= n || device >= kMaxDevices)
    return fail(KH_EINVAL, "device %d out of range", device);
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  HIP_TRY(hipSetDevice(device));
  device_cache(device).release();
  HIP_TRY(hipSetDevice(cur));
  return KH_OK;
}

extern "C" void kh_default_tuning(kh_tuning* t) {
  if (!t) return;
  // what the autotuner picks for the 10M-read metagenome at k = 21..99
  t->load_factor = 0.5f;
  t->bloom_bits = 2;
  t->bloom_lanes = 4;
  t->count_lanes = 2;
  t->tiles_per_block = 8;
  t->aggregate = 0;
  t->tails_overlap = 1;
  t->partitioned = 1;
}

extern "C" int kh_get_tuning(const kh_ctx* ctx, kh_tuning* out) {
  if (!ctx || !out) return fail(KH_EINVAL, "NULL argument");
  *out = ctx->tune;
  return KH_OK;
}

static bool lanes_ok(uint32_t j) { return j == 1 || j == 2 || j == 4; }

extern "C" int kh_set_tuning(kh_ctx* ctx, const kh_tuning* t) {
  if (!ctx || !t) return fail(KH_EINVAL, "NULL argument");
  if (!(t->load_factor >= 0.05f && t->load_factor < 0.95f))
    return fail(KH_EINVAL, "load_factor must be in [0.05, 0.95)");
  if (t->bloom_bits < 1 || t->bloom_bits > 64)
    return fail(KH_EINVAL, "bloom_bits must be in 1..64");
  if (!lanes_ok(t->bloom_lanes) || !(t->count_lanes == 0 || lanes_ok(t->count_lanes)))
    return fail(KH_EINVAL, "bloom_lanes must be 1, 2 or 4; count_lanes 0, 1, 2 or 4");
  if (t->tiles_per_block < 1 || t->tiles_per_block > 1024)
    return fail(KH_EINVAL, "tiles_per_block must be in 1..1024");
  if (t->aggregate > 1) return fail(KH_EINVAL, "aggregate must be 0 or 1");
  if (t->tails_overlap > 1) return fail(KH_EINVAL, "tails_overlap must be 0 or 1");
  if (t->partitioned > 1) return fail(KH_EINVAL, "partitioned must be 0 or 1");
  ctx->tune = *t;
  return KH_OK;
}

extern "C" int kh_autotune(kh_ctx* ctx, const kh_reads* reads, const kh_params* params,
                           const uint32_t* ks, int nk, void* hip_stream, int reps,
                           kh_tuning* out, kh_tune_report* report) {
  if (!ctx || !reads || !params || !ks || !out) return fail(KH_EINVAL, "NULL argument");
  if (nk < 1 || nk > kMaxK) return fail(KH_EINVAL, "nk must be in 1..%d", kMaxK);
  if (reps < 1) return fail(KH_EINVAL, "reps must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  kh_params p = *params;
  p.load_factor = 0.0f;  // the tuning under trial decides
  p.bloom_bits = 0;
  const kh_tuning start = ctx->tune;
  kh_tune_report rep{};
  // Time one setting: best of `reps` calls, tables freed at once.
  auto trial = [&](const kh_tuning& t, double* ms) -> int {
    ctx->tune = t;
    double best = 1e300;
    for (int r = 0; r < reps; ++r) {
      HIP_TRY(hipStreamSynchronize(s));
      const auto t0 = std::chrono::steady_clock::now();
      kh_table* outs[kMaxK] = {};
      const int rc = kh_count_multi_k(ctx, reads, &p, ks, nk, hip_stream, outs);
      if (rc != KH_OK) return rc;
      const auto t1 = std::chrono::steady_clock::now();
      for (int i = 0; i < nk; ++i) kh_table_free(outs[i]);
      best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    ++rep.trials;
    *ms = best;
    return KH_OK;
  };
  double best_ms = 0;
  kh_tuning best = start;
  int rc = trial(start, &best_ms);
  if (rc != KH_OK) {
    ctx->tune = start;
    return rc;
  }
  rep.start_ms = best_ms;
  // one field at a time; a change is kept if it saves at least 1 %
  auto field = [&](auto set, std::initializer_list<double> values) -> int {
    for (double v : values) {
      kh_tuning t = best;
      set(t, v);
      if (std::memcmp(&t, &best, sizeof t) == 0) continue;
      double ms = 0;
      const int r = trial(t, &ms);
      if (r == KH_ENOMEM) {
        ++rep.skipped;
        continue;
      }
      if (r != KH_OK) return r;
      if (ms < 0.99 * best_ms) {
        best = t;
        best_ms = ms;
      }
    }
    return KH_OK;
  };
  rc = field([](kh_tuning& t, double v) { t.partitioned = (uint32_t)v; }, {1, 0});
  // the remaining fields shape the single-table path only
  const bool single = !best.partitioned;
  if (rc == KH_OK && single)
    rc = field([](kh_tuning& t, double v) { t.count_lanes = (uint32_t)v; }, {4, 2, 1, 0});
  if (rc == KH_OK && single && params->use_bloom)
    rc = field([](kh_tuning& t, double v) { t.bloom_lanes = (uint32_t)v; }, {4, 2, 1});
  if (rc == KH_OK && single)
    rc = field([](kh_tuning& t, double v) { t.tiles_per_block = (uint32_t)v; }, {1, 2, 4, 8});
  if (rc == KH_OK && single)
    rc = field([](kh_tuning& t, double v) { t.load_factor = (float)v; },
               {0.6, 0.5, 0.4, 0.3});
  if (rc == KH_OK && single && params->use_bloom)
    rc = field([](kh_tuning& t, double v) { t.bloom_bits = (uint32_t)v; }, {4, 3, 2, 6});
  if (rc == KH_OK && single)
    rc = field([](kh_tuning& t, double v) { t.aggregate = (uint32_t)v; }, {0, 1});
  if (rc == KH_OK && single && nk > 1)
    rc = field([](kh_tuning& t, double v) { t.tails_overlap = (uint32_t)v; }, {1, 0});
  if (rc != KH_OK) {
    ctx->tune = start;
    return rc;
  }
  ctx->tune = best;
  rep.best_ms = best_ms;
  *out = best;
  if (report) *report = rep;
  return KH_OK;
}

// The case a stored tuning applies to: device, k set, read set size, Bloom
// setting and key-space parts.
static int tune_case(kh_ctx* ctx, const kh_reads* r, const kh_params& p, const uint32_t* ks,
                     int nk, hipStream_t s, std::string* key) {
  int64_t bases = 0;
  if (r->n_reads > 0) {
    if (!r->offsets) return fail(KH_EINVAL, "offsets is NULL");
    if (r->on_device) {
      HIP_TRY(hipMemcpyAsync(&bases, r->offsets + r->n_reads, sizeof bases,
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
    } else {
      bases = r->offsets[r->n_reads];
    }
  }
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, ctx->device));
  char arch[64];
  std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
  for (char* c = arch; *c; ++c)
    if (*c == ':' || *c == ' ') *c = '_';
  std::string kl;
  for (int i = 0; i < nk; ++i) kl += (i ? "," : "") + std::to_string(ks[i]);
  char buf[512];
  std::snprintf(buf, sizeof buf, "arch=%s cus=%d ks=%s reads=%lld bases=%lld bloom=%d parts=%u",
                arch, prop.multiProcessorCount, kl.c_str(), (long long)r->n_reads,
                (long long)bases, p.use_bloom ? 1 : 0,
                p.owner_shards > 1 ? p.owner_shards : 1u);
  *key = buf;
  return KH_OK;
}

extern "C" int kh_autotune_cached(kh_ctx* ctx, const kh_reads* reads, const kh_params* params,
                                  const uint32_t* ks, int nk, void* hip_stream, int reps,
                                  const char* cache_path, kh_tuning* out,
                                  kh_tune_report* report, int* hit) {
  if (hit) *hit = 0;
  if (!ctx || !reads || !params || !ks || !out || !cache_path)
    return fail(KH_EINVAL, "NULL argument");
  if (nk < 1 || nk > kMaxK) return fail(KH_EINVAL, "nk must be in 1..%d", kMaxK);
  KH_TRY(set_device(ctx));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::string key;
  KH_TRY(tune_case(ctx, reads, *params, ks, nk, s, &key));
  bool found = false;
  kh_tuning t{};
  if (FILE* f = std::fopen(cache_path, "r")) {
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
      const char* bar = std::strstr(line, " | ");
      if (!bar || std::string(line, bar - line) != key) continue;
      kh_tuning u{};
      if (std::sscanf(bar + 3,
                      "load_factor=%f bloom_bits=%u bloom_lanes=%u count_lanes=%u "
                      "tiles_per_block=%u aggregate=%u tails_overlap=%u partitioned=%u",
                      &u.load_factor, &u.bloom_bits, &u.bloom_lanes, &u.count_lanes,
                      &u.tiles_per_block, &u.aggregate, &u.tails_overlap,
                      &u.partitioned) == 8) {
        t = u;
        found = true;
      }
    }
    std::fclose(f);
  }
  if (found) {
    KH_TRY(kh_set_tuning(ctx, &t));
    *out = t;
    if (report) *report = kh_tune_report{};
    if (hit) *hit = 1;
    return KH_OK;
  }
  KH_TRY(kh_autotune(ctx, reads, params, ks, nk, hip_stream, reps, out, report));
  if (FILE* f = std::fopen(cache_path, "a")) {
    std::fprintf(f,
                 "%s | load_factor=%.4f bloom_bits=%u bloom_lanes=%u count_lanes=%u "
                 "tiles_per_block=%u aggregate=%u tails_overlap=%u partitioned=%u\n",
                 key.c_str(), out->load_factor, out->bloom_bits, out->bloom_lanes,
                 out->count_lanes, out->tiles_per_block, out->aggregate, out->tails_overlap,
                 out->partitioned);
    std::fclose(f);
  }
  return KH_OK;
}

extern "C" int kh_set_timing(kh_ctx* ctx, int enable) {
  if (!ctx) return fail(KH_EINVAL, "ctx is NULL");
  ctx->timing = enable ? 1 : 0;
  return KH_OK;
}

extern "C" int kh_last_timing(const kh_ctx* ctx, float ms[6]) {
  if (!ctx || !ms) return fail(KH_EINVAL, "NULL argument");
  std::memcpy(ms, ctx->last_ms, sizeof ctx->last_ms);
  return KH_OK;
}

extern "C" int kh_last_stats(const kh_ctx* ctx, uint64_t out[12]) {
  if (!ctx || !out) return fail(KH_EINVAL, "NULL argument");
  std::memcpy(out, ctx->last_stats, sizeof ctx->last_stats);
  return KH_OK;
}

extern "C" int kh_last_graphed(const kh_ctx* ctx, int* graphed) {
  if (!ctx || !graphed) return fail(KH_EINVAL, "NULL argument");
  *graphed = ctx->last_graphed;
  return KH_OK;
}

extern "C" int kh_last_k_report(const kh_ctx* ctx, int i, float ms[6],
                                uint64_t stats[12]) {
  if (!ctx) return fail(KH_EINVAL, "ctx is NULL");
  if (i < 0 || i >= kMaxK) return fail(KH_EINVAL, "index %d out of range", i);
  if (ms) std::memcpy(ms, ctx->k_ms[i], sizeof ctx->k_ms[i]);
  if (stats) std::memcpy(stats, ctx->k_stats[i], sizeof ctx->k_stats[i]);
  return KH_OK;
}

extern "C" int kh_count(kh_ctx* ctx, const kh_reads* reads,
                        const kh_params* params, void* stream, kh_table** out) {
  if (!ctx || !out) return fail(KH_EINVAL, "ctx or out is NULL");
  *out = nullptr;
  KH_TRY(check_params(params));
  KH_TRY(set_device(ctx));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Packed pk(&ctx->pool);
  start_timing(ctx);
  mark(ctx, 0, s);
  // host reads with the Bloom screen: uploaded in chunks during pass A
  KH_TRY(pack_reads(ctx, reads, *params, s, pk, params->use_bloom != 0));
  mark(ctx, 1, s);
  const int rc = count_packed(ctx, pk, *params, s, out);
  if (rc == KH_OK) accumulate_phases(ctx, 0, 0);
  return rc;
}

extern "C" int kh_count_multi_k(kh_ctx* ctx, const kh_reads* reads,
                                const kh_params* params, const uint32_t* ks,
                                int nk, void* stream, kh_table** outs) {
  if (!ctx || !outs || !ks) return fail(KH_EINVAL, "NULL argument");
  if (nk < 1 || nk > 8) return fail(KH_EINVAL, "nk must be in 1..8");
  for (int i = 0; i < nk; ++i) outs[i] = nullptr;
  KH_TRY(check_params(params));
  for (int i = 0; i < nk; ++i) {
    kh_params q = *params;
    q.k = ks[i];
    KH_TRY(check_params(&q));
  }
  KH_TRY(set_device(ctx));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Packed pk(&ctx->pool);
  start_timing(ctx);
  mark(ctx, 0, s);
  // host reads with the Bloom screen: the batched path uploads them in
  // chunks, each chunk's Bloom pass overlapping the next chunk's copy
  const bool owned = owned_applies(ctx);
  KH_TRY(pack_reads(ctx, reads, *params, s, pk, nk > 1 && params->use_bloom && !owned));
  mark(ctx, 1, s);
  if (nk > 1 && !owned) {
    const int rc = count_multi_batched(ctx, pk, *params, ks, nk, s, outs);
    ctx->cur_k = 0;
    if (rc != KH_ENOMEM) {
      if (rc == KH_OK) accumulate_phases(ctx, 0, 0);
      return rc;
    }
    // every table at once does not fit: count the k one after another
    HIP_TRY(hipDeviceSynchronize());
    start_timing(ctx);
  }
  KH_TRY(finish_pack(ctx, pk, s));
  for (int i = 0; i < nk; ++i) {
    kh_params q = *params;
    q.k = ks[i];
    ctx->cur_k = i;
    int rc = count_packed(ctx, pk, q, s, &outs[i]);
    if (rc != KH_OK) {
      for (int j = 0; j < i; ++j) {
        kh_table_free(outs[j]);
        outs[j] = nullptr;
      }
      return rc;
    }
  }
  ctx->cur_k = 0;
  accumulate_phases(ctx, 0, 0);  // the shared pack is booked on the first k
  return KH_OK;
}

extern "C" int kh_table_info(const kh_table* t, uint32_t* k, uint32_t* W,
                             int64_t* n_rows, uint64_t* n_windows) {
  if (!t) return fail(KH_EINVAL, "table is NULL");
  if (k) *k = t->k;
  if (W) *W = t->W;
  if (n_rows) *n_rows = t->n_rows;
  if (n_windows) *n_windows = t->n_windows;
  return KH_OK;
}

extern "C" int kh_table_export(const kh_table* t, uint64_t* keys,
                               uint32_t* counts, uint32_t* ext, uint8_t* codes,
                               int dst_on_device, void* stream) {
  if (!t) return fail(KH_EINVAL, "table is NULL");
  if (t->n_rows == 0) return KH_OK;
  HIP_TRY(hipSetDevice(t->ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const uint64_t n = (uint64_t)t->n_rows;
  if (keys) HIP_TRY(hipMemcpyAsync(keys, t->keys, n * t->W * 8, kind, s));
  if (counts) HIP_TRY(hipMemcpyAsync(counts, t->counts, n * 4, kind, s));
  if (ext) HIP_TRY(hipMemcpyAsync(ext, t->ext, n * 32, kind, s));
  if (codes) HIP_TRY(hipMemcpyAsync(codes, t->codes, n * 2, kind, s));
  HIP_TRY(hipStreamSynchronize(s));
  return KH_OK;
}

extern "C" int kh_table_device_rows(const kh_table* t, const uint64_t** keys,
                                    const uint32_t** counts, const uint32_t** ext,
                                    const uint8_t** codes) {
  if (!t) return fail(KH_EINVAL, "table is NULL");
  if (keys) *keys = t->keys;
  if (counts) *counts = t->counts;
  if (ext) *ext = t->ext;
  if (codes) *codes = t->codes;
  return KH_OK;
}

extern "C" int kh_table_free(kh_table* t) {
  if (!t) return KH_OK;
  if (t->ctx) {
    Pool& pl = t->ctx->pool;
    std::lock_guard<std::recursive_mutex> lk(pl.mu);
    t->ctx->live.erase(t);
    pl.put(t->keys);
    pl.put(t->counts);
    pl.put(t->ext);
    pl.put(t->codes);
  }
  delete t;
  return KH_OK;
}
