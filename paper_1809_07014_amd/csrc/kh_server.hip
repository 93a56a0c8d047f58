// Serving engine: continuous batching of read batches from many samples.
//
// A worker thread owns the device.  Submitted requests wait in a queue and
// are admitted in arrival order while fewer than `max_active` are running
// and the device memory in use (the pool's blocks minus those free for
// reuse) plus the expected needs of the running requests stays under 60 % of
// the HBM budget (85 % of the device when none is given); the oldest request
// always runs.  A launch that cannot reserve its memory counts nothing and
// is retried with the oldest request alone.  Every launch is built from chunks (`chunk_reads` reads) of several admitted
// requests (round robin, up to `batch_bases` bases; in plain mode one chunk
// of the oldest request): each chunk is packed into its sample's resident
// arena of packed reads, and one counting launch per k covers the tiles of
// all chunks, each tile updating the table of its own sample (per-tile
// descriptors).  Requests that arrive while others run join the next launch.
// A sample's tables (one per k) stay resident and grow by rehash before a
// launch that is expected to fill them past 70 %; windows that still find
// a table full (probe limit) are listed and replayed into the grown table
// after the launch.  kh_server_finalize turns a sample's
// tables into sorted rows with the same tail as kh_count (classify, exact
// heavy-hitter recount over the sample's arena, sort, gather) and frees the
// sample.  Counting is exact: the Bloom screen is not used (a k-mer's
// occurrences may span batches), and a table is a sum of per-window updates,
// so its final state does not depend on how the batches were grouped (the
// paper's Section II-A, Use case 1).
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <memory>
#include <thread>
#include <vector>

#include "kh_host.hpp"

using namespace kh;
using Clock = std::chrono::steady_clock;

namespace {

struct Arena {  // packed reads of one sample, append-only
  Buf<uint64_t> bases, hq, bad, st;
  int64_t len = 0;  // positions in use (next chunk starts at a multiple of 64)
  int64_t cap = 0;  // positions allocated
  std::vector<std::pair<int64_t, int64_t>> chunks;  // [start, end) per chunk
  explicit Arena(Pool* p) : bases(p), hq(p), bad(p), st(p) {}
};

struct SampleState {
  uint64_t id;
  Arena arena;
  Buf<uint8_t> table[kMaxK];
  uint64_t cap[kMaxK] = {};
  uint64_t claimed[kMaxK] = {};
  uint64_t windows[kMaxK] = {};
  uint64_t pending_bases = 0;  // bases of its launches enqueued, not finished
  int open_requests = 0;
  int error = KH_OK;
  std::string error_msg;
  SampleState(Pool* p, uint64_t sid) : id(sid), arena(p) {
    for (auto& b : table) b.pool = p;
  }
};

struct Request {
  uint64_t ticket = 0, sample = 0;
  kh_reads reads{};
  int64_t next = 0;      // first read not yet taken into a launch
  int64_t inflight = 0;  // chunks taken and not yet counted
  uint64_t reserve = 0;  // device bytes still expected for it (admission)
  double reserve_per_base = 0;  // reserve spent per base taken
  Clock::time_point t_submit, t_done;
  bool done = false;
  int status = KH_OK;
  std::string msg;  // the failure's message (status != KH_OK)
};

struct FinalizeCmd {
  uint64_t sample = 0;
  kh_table** outs = nullptr;
  bool done = false;
  int status = KH_OK;
  std::string msg;
};

struct Take {
  Request* r;
  SampleState* smp;
  int64_t r0, r1;      // reads [r0, r1) of the request
  int64_t start = 0;   // arena position of the packed chunk
  int64_t n = 0;       // bases
  int slot = 0;        // index of the sample among this launch's samples
  uint64_t reserve = 0;  // admission reserve the chunk took from its request
};

// Pinned host memory (hipHostMalloc), grown on demand.
struct PinnedBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// One of the two staging sets: device buffers the copy stream uploads a
// launch's chunks into, and the pinned host buffers of that launch (rebased
// offsets, tile descriptors, counters read back).  Launches alternate sets,
// so a set is reused only after the launch before the previous one has
// finished.
struct StageSet {
  Buf<uint8_t> seq, qual;
  Buf<int64_t> off;
  int64_t bases_cap = 0, reads_cap = 0;
  PinnedBuf hoff, hdesc, hctr;
  explicit StageSet(Pool* p) : seq(p), qual(p), off(p) {}
};

// A launch from staging to finish.
struct Launch {
  std::vector<Take> takes;
  std::vector<SampleState*> smps;
  std::vector<int64_t> base_at, off_at;  // each chunk's place in the staging set
  std::vector<uint64_t> smp_bases;       // bases of each sample in this launch
  bool enqueued = false;
  int set = 0;
  uint64_t nwmax = 0;                    // windows (tile-rounded): overflow capacity
  size_t nctr = 0;
  // counters: [2 (k nsm + j)] claimed / windows of sample j at k, then the
  // overflow count of every k, then a status block (kCtrCount words)
  Buf<unsigned long long> ctr;
  Buf<TileDesc> ddesc;                   // descriptors of every k, back to back
  Buf<uint64_t> ovf[kMaxK];              // overflow list of every k
  std::vector<TileDesc> descs[kMaxK];
  std::vector<int> desc_slot[kMaxK];
  size_t desc_at[kMaxK] = {};
  explicit Launch(Pool* p) : ctr(p), ddesc(p) {
    for (auto& b : ovf) b.pool = p;
  }
};

// Internal result of a launch that could not reserve its device memory
// before counting anything (the worker retries it smaller).
constexpr int kNoRoom = -100;

inline int64_t align64(int64_t x) { return (x + 63) & ~int64_t(63); }

}  // namespace

struct kh_server {
  kh_ctx* ctx = nullptr;
  kh_params params{};
  uint32_t ks[kMaxK] = {};
  int nk = 0;
  kh_server_config cfg{};
  hipStream_t stream = nullptr;  // packing, counting, growth, finalize
  hipStream_t copy = nullptr;    // uploads of the next launch's chunks
  hipEvent_t copy_ev[2] = {}, done_ev[2] = {};
  std::unique_ptr<StageSet> stage[2];
  uint64_t seq_no = 0;           // launches staged
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<Request*> pending;
  std::vector<Request*> active;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
  std::unordered_map<uint64_t, std::unique_ptr<SampleState>> samples;
  std::deque<FinalizeCmd*> finalize_q;
  // statistics
  uint64_t n_done = 0, n_launches = 0, n_rehash = 0, max_active_seen = 0;
  uint64_t n_replayed = 0;
  uint64_t force_slots = 0;  // test hook: fixed first size, growth by replay only
  double pack_s = 0, grow_s = 0;
  // admission: device bytes expected per base of a request, and the sum of
  // the admitted requests' unspent reserves
  uint64_t reserved = 0;
  bool solo_next = false;   // next launch: the oldest request only
  uint64_t n_retried = 0;   // launches that did not fit and were retried
  double windows_total = 0.0, busy_s = 0.0;
};

// ------------------------------------------------------------ device work --

static uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

static int arena_reserve(kh_ctx* ctx, Arena& a, int64_t need, hipStream_t s) {
  if (need <= a.cap) return KH_OK;
  int64_t cap = std::max<int64_t>(need, std::max<int64_t>(a.cap * 2, 1 << 20));
  cap = (int64_t)pow2_at_least((uint64_t)cap);
  const int64_t bw = cap / 32 + 4, pw = cap / 64 + 4;
  Buf<uint64_t> nb(&ctx->pool), nh(&ctx->pool), nx(&ctx->pool), ns(&ctx->pool);
  KH_TRY(nb.alloc(bw));
  KH_TRY(nh.alloc(pw));
  KH_TRY(nx.alloc(pw));
  KH_TRY(ns.alloc(pw));
  launch_fill_u64(nb.p, bw, 0ull, s);
  launch_fill_u64(nh.p, pw, 0ull, s);
  launch_fill_u64(nx.p, pw, ~0ull, s);  // unused positions are not bases
  launch_fill_u64(ns.p, pw, 0ull, s);
  if (a.len > 0) {
    HIP_TRY(hipMemcpyAsync(nb.p, a.bases.p, (a.len / 32 + 2) * 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(nh.p, a.hq.p, (a.len / 64 + 1) * 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(nx.p, a.bad.p, (a.len / 64 + 1) * 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(ns.p, a.st.p, (a.len / 64 + 1) * 8, hipMemcpyDeviceToDevice, s));
  }
  // the old planes go back to the pool now: a block reused from it is only
  // ever used by work queued later on the same stream
  std::swap(a.bases.p, nb.p);
  std::swap(a.hq.p, nh.p);
  std::swap(a.bad.p, nx.p);
  std::swap(a.st.p, ns.p);
  a.cap = cap;
  return KH_OK;
}

// Grow table ki of a sample to at least min_cap slots (and at least twice
// its size) by rehash.  Tables are sized for a load of at most one half
// after growth; a launch that still fills one up hands the windows that
// found no slot to the replay.
static int table_grow_(kh_server* S, SampleState& smp, int ki, uint64_t min_cap,
                       unsigned long long* status, hipStream_t s);
static int table_grow(kh_server* S, SampleState& smp, int ki, uint64_t min_cap,
                      unsigned long long* status, hipStream_t s) {
  const auto t0 = Clock::now();
  const int rc = table_grow_(S, smp, ki, min_cap, status, s);
  S->grow_s += std::chrono::duration<double>(Clock::now() - t0).count();
  return rc;
}

// The rehash raises kStatusProbeLimit in status[kCtrStatus] if a key finds
// no slot (it cannot in a table twice as large); the launch reads it back
// with its counters.
static int table_grow_(kh_server* S, SampleState& smp, int ki, uint64_t min_cap,
                       unsigned long long* status, hipStream_t s) {
  const uint32_t k = S->ks[ki];
  const SlotLayout lay = slot_layout(table_chunks(k));
  // power-of-two sizes, so that a table given up by one sample fits the
  // next one that grows to that size
  uint64_t cap = std::max<uint64_t>(min_cap, 2 * smp.cap[ki]);
  cap = pow2_at_least(cap);
  if (cap >= (1ull << 32)) return fail(KH_ENOMEM, "sample table exceeds 2^32 slots");
  Buf<uint8_t> nt(&S->ctx->pool);
  KH_TRY(nt.alloc(cap * lay.stride));
  launch_fill_u64(reinterpret_cast<uint64_t*>(nt.p), cap * lay.stride / 8, 0ull, s);
  if (smp.cap[ki] > 0) {
    launch_rehash(smp.table[ki].p, smp.cap[ki], nt.p, cap, k, status, s);
    HIP_TRY(hipGetLastError());
    ++S->n_rehash;
  }
  std::swap(smp.table[ki].p, nt.p);
  smp.cap[ki] = cap;
  return KH_OK;
}

static int table_reserve(kh_server* S, SampleState& smp, int ki, uint64_t windows,
                         unsigned long long* status, hipStream_t s) {
  // keys expected after the launch: those held, plus its windows at the
  // sample's rate of new keys per window so far (1, every window a new key,
  // before any is booked: a sample's first chunks cover little of its
  // genomes; the rate falls as coverage builds, so the running mean
  // over-estimates; a launch that still overflows is replayed)
  const double rate =
      smp.windows[ki] ? std::max(0.02, (double)smp.claimed[ki] / (double)smp.windows[ki]) : 1.0;
  const double expect = (double)smp.claimed[ki] + rate * (double)windows;
  if (S->force_slots)
    return smp.cap[ki] ? KH_OK : table_grow(S, smp, ki, S->force_slots, status, s);
  if (smp.cap[ki] == 0)
    return table_grow(S, smp, ki, std::max<uint64_t>(1 << 20, (uint64_t)(expect / 0.5)),
                      status, s);
  if (expect > 0.7 * (double)smp.cap[ki])
    return table_grow(S, smp, ki, (uint64_t)(expect / 0.5), status, s);
  return KH_OK;
}

// ------------------------------------------------------------- launches --
//
// A launch goes through three steps.  stage_launch copies its chunks' bases,
// qualities and rebased offsets into one of two device staging sets on the
// copy stream.  enqueue_launch reserves arena room and table growth, packs
// the chunks from the staging set into their samples' arenas once the copy
// has landed, runs one counting pass per k over the tiles of every chunk and
// copies the launch's counters back into pinned host memory, all on the
// compute stream without waiting.  finish_launch waits for that copy, books
// the counts, and replays windows that found a table full.  The worker
// stages and enqueues launch n + 1 before it finishes launch n, so the next
// upload overlaps the current counting passes; plain mode finishes every
// launch before building the next.

// Grow a pinned host buffer (no launch that used the old one is in flight).
static int pinned_reserve(PinnedBuf& b, size_t bytes) {
  if (bytes <= b.cap) return KH_OK;
  const size_t cap = std::max(bytes, 2 * b.cap);
  if (b.p) (void)hipHostFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  HIP_TRY(hipHostMalloc(&b.p, cap, hipHostMallocDefault));
  b.cap = cap;
  return KH_OK;
}

static int stage_launch(kh_server* S, Launch& L) {
  const auto t0 = Clock::now();
  L.set = (int)(S->seq_no++ & 1);
  StageSet& st = *S->stage[L.set];
  // the set's last upload has landed (it has, unless that launch was handed
  // back before packing): its pinned offsets may be rewritten
  HIP_TRY(hipEventSynchronize(S->copy_ev[L.set]));
  int64_t nb = 0, nr = 0;
  for (Take& t : L.takes) {  // each chunk's bases at a 64-byte boundary
    const int64_t* ho = t.r->reads.offsets;
    t.n = ho[t.r1] - ho[t.r0];
    L.base_at.push_back(nb);
    L.off_at.push_back(nr);
    nb += align64(t.n);
    nr += t.r1 - t.r0 + 1;
  }
  if (nb > st.bases_cap || nr > st.reads_cap) {
    // rare: the old buffers may be named by queued copies or packs
    HIP_TRY(hipStreamSynchronize(S->copy));
    HIP_TRY(hipStreamSynchronize(S->stream));
    st.bases_cap = std::max<int64_t>(nb, 2 * st.bases_cap);
    st.reads_cap = std::max<int64_t>(nr, 2 * st.reads_cap);
    KH_TRY(st.seq.alloc((uint64_t)st.bases_cap));
    KH_TRY(st.qual.alloc((uint64_t)st.bases_cap));
    KH_TRY(st.off.alloc((uint64_t)st.reads_cap));
  }
  KH_TRY(pinned_reserve(st.hoff, (size_t)nr * 8));
  int64_t* ho_pin = static_cast<int64_t*>(st.hoff.p);
  for (size_t i = 0; i < L.takes.size(); ++i) {
    const Take& t = L.takes[i];
    const int64_t* ho = t.r->reads.offsets;
    const int64_t a = ho[t.r0];
    for (int64_t j = 0; j <= t.r1 - t.r0; ++j) ho_pin[L.off_at[i] + j] = ho[t.r0 + j] - a;
    if (t.n > 0) {
      HIP_TRY(hipMemcpyAsync(st.seq.p + L.base_at[i], t.r->reads.seq + a, t.n,
                             hipMemcpyHostToDevice, S->copy));
      HIP_TRY(hipMemcpyAsync(st.qual.p + L.base_at[i], t.r->reads.qual + a, t.n,
                             hipMemcpyHostToDevice, S->copy));
    }
  }
  HIP_TRY(hipMemcpyAsync(st.off.p, ho_pin, (size_t)nr * 8, hipMemcpyHostToDevice, S->copy));
  HIP_TRY(hipEventRecord(S->copy_ev[L.set], S->copy));
  S->pack_s += std::chrono::duration<double>(Clock::now() - t0).count();
  return KH_OK;
}

static int enqueue_launch(kh_server* S, Launch& L) {
  kh_ctx* ctx = S->ctx;
  hipStream_t s = S->stream;
  StageSet& st = *S->stage[L.set];
  for (Take& t : L.takes) {
    auto it = std::find(L.smps.begin(), L.smps.end(), t.smp);
    t.slot = (int)(it - L.smps.begin());
    if (it == L.smps.end()) L.smps.push_back(t.smp);
  }
  const size_t nsm = L.smps.size(), nk = (size_t)S->nk;
  L.nctr = 2 * nsm * nk + nk + kCtrCount;
  KH_TRY(L.ctr.alloc(L.nctr));
  launch_fill_u64(reinterpret_cast<uint64_t*>(L.ctr.p), L.nctr, 0ull, s);
  unsigned long long* status = L.ctr.p + 2 * nsm * nk + nk;
  // ---- reserve first: arena room for every chunk and table growth for
  // every sample and k, so that a launch that does not fit counts nothing.
  // A table is sized for this launch's windows and those of the sample's
  // launches still in flight, whose keys are not booked yet.
  L.smp_bases.assign(nsm, 0);
  {
    std::vector<int64_t> end(nsm);
    for (size_t j = 0; j < nsm; ++j) end[j] = L.smps[j]->arena.len;
    for (Take& t : L.takes) {
      t.start = align64(end[t.slot]);
      end[t.slot] = t.start + t.n;
      L.smp_bases[t.slot] += (uint64_t)t.n;
    }
    for (size_t j = 0; j < nsm; ++j) {
      int rc = arena_reserve(ctx, L.smps[j]->arena, end[j] + 256, s);
      for (int ki = 0; rc == KH_OK && ki < S->nk; ++ki)
        rc = table_reserve(S, *L.smps[j], ki, L.smp_bases[j] + L.smps[j]->pending_bases,
                           status, s);
      if (rc == KH_ENOMEM) return kNoRoom;
      KH_TRY(rc);
    }
  }
  // ---- pack every chunk from the staging set into its sample's arena
  HIP_TRY(hipStreamWaitEvent(s, S->copy_ev[L.set], 0));
  for (size_t i = 0; i < L.takes.size(); ++i) {
    Take& t = L.takes[i];
    Arena& ar = t.smp->arena;
    if (t.n > 0) {
      PackArgs pa{};
      pa.seq = st.seq.p + L.base_at[i];
      pa.qual = st.qual.p + L.base_at[i];
      pa.offsets = st.off.p + L.off_at[i];
      pa.n_reads = t.r1 - t.r0;
      pa.n = t.n;
      pa.qual_offset = (int)S->params.qual_offset;
      pa.qual_cutoff = (int)S->params.qual_cutoff;
      pa.bases = ar.bases.p + t.start / 32;
      pa.hq = ar.hq.p + t.start / 64;
      pa.bad = ar.bad.p + t.start / 64;
      pa.st = ar.st.p + t.start / 64;
      pa.plane_words = (t.n + 63) / 64;
      pa.ctr = ctx->ctr;
      launch_pack(pa, s);
      HIP_TRY(hipGetLastError());
    }
    ar.chunks.emplace_back(t.start, t.start + t.n);
    ar.len = t.start + t.n;
  }
  // ---- tile descriptors of every k (one upload from pinned memory), then
  // one counting pass per k; windows that find a full table go to the k's
  // overflow list
  L.nwmax = 0;
  for (Take& t : L.takes) L.nwmax += (uint64_t)((t.n + kTile - 1) / kTile) * kTile;
  if (L.nwmax > 0) {
    size_t total = 0;
    for (size_t ki = 0; ki < nk; ++ki) {
      KH_TRY(L.ovf[ki].alloc(L.nwmax));
      L.desc_at[ki] = total;
      L.descs[ki].clear();
      L.desc_slot[ki].clear();
      for (Take& t : L.takes) {
        Arena& ar = t.smp->arena;
        for (int64_t p0 = t.start; p0 < t.start + t.n; p0 += kTile) {
          TileDesc d{};
          d.bases = ar.bases.p;
          d.hq = ar.hq.p;
          d.bad = ar.bad.p;
          d.st = ar.st.p;
          d.base_words = ar.cap / 32 + 4;
          d.plane_words = ar.cap / 64 + 4;
          d.p0 = p0;
          d.hi = t.start + t.n;
          d.table = t.smp->table[ki].p;
          d.capacity = t.smp->cap[ki];
          d.counters = L.ctr.p + 2 * (ki * nsm + (size_t)t.slot);
          d.overflow = L.ovf[ki].p;
          d.overflow_n = L.ctr.p + 2 * nsm * nk + ki;
          d.overflow_cap = L.nwmax;
          L.descs[ki].push_back(d);
          L.desc_slot[ki].push_back(t.slot);
        }
      }
      total += L.descs[ki].size();
    }
    KH_TRY(pinned_reserve(st.hdesc, total * sizeof(TileDesc)));
    TileDesc* hd = static_cast<TileDesc*>(st.hdesc.p);
    for (size_t ki = 0; ki < nk; ++ki)
      std::memcpy(hd + L.desc_at[ki], L.descs[ki].data(), L.descs[ki].size() * sizeof(TileDesc));
    KH_TRY(L.ddesc.alloc(total));
    HIP_TRY(hipMemcpyAsync(L.ddesc.p, hd, total * sizeof(TileDesc), hipMemcpyHostToDevice, s));
    for (size_t ki = 0; ki < nk; ++ki) {
      WindowArgs wa{};
      wa.k = S->ks[ki];
      wa.ctr = status;
      wa.lanes = (int)ctx->tune.count_lanes;
      wa.tiles = L.ddesc.p + L.desc_at[ki];
      wa.n_tiles = (int64_t)L.descs[ki].size();
      wa.count_windows = 1;
      launch_windows(wa, 0, s);
      HIP_TRY(hipGetLastError());
    }
  }
  // ---- the launch's counters back in one copy
  KH_TRY(pinned_reserve(st.hctr, L.nctr * 8));
  HIP_TRY(hipMemcpyAsync(st.hctr.p, L.ctr.p, L.nctr * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(S->done_ev[L.set], s));
  for (size_t j = 0; j < nsm; ++j) L.smps[j]->pending_bases += L.smp_bases[j];
  L.enqueued = true;
  return KH_OK;
}

static int finish_launch(kh_server* S, Launch& L) {
  hipStream_t s = S->stream;
  StageSet& st = *S->stage[L.set];
  const size_t nsm = L.smps.size(), nk = (size_t)S->nk;
  if (L.enqueued)
    for (size_t j = 0; j < nsm; ++j) L.smps[j]->pending_bases -= L.smp_bases[j];
  HIP_TRY(hipEventSynchronize(S->done_ev[L.set]));
  const unsigned long long* hc = static_cast<const unsigned long long*>(st.hctr.p);
  if (hc[2 * nsm * nk + nk + kCtrStatus] & kStatusProbeLimit)
    return fail(KH_EDEVICE, "a table rehash lost a key");
  std::vector<uint64_t> n_ovf(nk);
  for (size_t ki = 0; ki < nk; ++ki) {
    for (size_t j = 0; j < nsm; ++j) {
      L.smps[j]->claimed[ki] += hc[2 * (ki * nsm + j)];
      L.smps[j]->windows[ki] += hc[2 * (ki * nsm + j) + 1];
      S->windows_total += (double)hc[2 * (ki * nsm + j) + 1];
    }
    n_ovf[ki] = hc[2 * nsm * nk + ki];
  }
  // ---- some tables filled up: grow them, then replay their windows (the
  // compute stream may already hold the next launch, which ran on the old
  // tables; the rehash comes after it and carries its counts along)
  std::vector<uint64_t> entries;
  std::vector<unsigned long long> cc(2 * nsm + kCtrCount);
  unsigned long long* status = L.ctr.p + 2 * nsm * nk + nk;
  for (size_t ki = 0; ki < nk; ++ki) {
    if (n_ovf[ki] == 0) continue;
    entries.resize(n_ovf[ki]);
    HIP_TRY(hipMemcpyAsync(entries.data(), L.ovf[ki].p, n_ovf[ki] * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<uint64_t> per(nsm, 0);
    for (uint64_t e : entries) per[L.desc_slot[ki][e >> 10]]++;
    for (size_t j = 0; j < nsm; ++j)
      if (per[j])
        KH_TRY(table_grow(S, *L.smps[j], (int)ki,
                          (uint64_t)((double)(L.smps[j]->claimed[ki] + per[j]) / 0.5), status,
                          s));
    for (size_t d = 0; d < L.descs[ki].size(); ++d) {
      SampleState* smp = L.smps[L.desc_slot[ki][d]];
      L.descs[ki][d].table = smp->table[ki].p;
      L.descs[ki][d].capacity = smp->cap[ki];
    }
    TileDesc* hd = static_cast<TileDesc*>(st.hdesc.p) + L.desc_at[ki];
    std::memcpy(hd, L.descs[ki].data(), L.descs[ki].size() * sizeof(TileDesc));
    HIP_TRY(hipMemcpyAsync(L.ddesc.p + L.desc_at[ki], hd, L.descs[ki].size() * sizeof(TileDesc),
                           hipMemcpyHostToDevice, s));
    launch_fill_u64(reinterpret_cast<uint64_t*>(L.ctr.p + 2 * ki * nsm), 2 * nsm, 0ull, s);
    launch_replay(L.ddesc.p + L.desc_at[ki], L.ovf[ki].p, n_ovf[ki], S->ks[ki], s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(cc.data(), L.ctr.p + 2 * ki * nsm, 2 * nsm * 8,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(cc.data() + 2 * nsm, status, kCtrCount * 8,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (cc[2 * nsm + kCtrStatus] & kStatusProbeLimit)
      return fail(KH_EDEVICE, "a table rehash lost a key");
    for (size_t j = 0; j < nsm; ++j) L.smps[j]->claimed[ki] += cc[2 * j];
    S->n_replayed += n_ovf[ki];
  }
  ++S->n_launches;
  return KH_OK;
}

// Device bytes a finalize may need at most, with rows bounded by the keys
// held: the exported rows of every k, plus the largest per-k working set
// (classify output at 12 B per slot, sort buffers, full-key sort keys).
static uint64_t finalize_bytes(kh_server* S, const SampleState& smp) {
  uint64_t rows = 0, work = 0;
  for (int ki = 0; ki < S->nk; ++ki) {
    const uint64_t W = (S->ks[ki] + 31) / 32;
    rows += smp.claimed[ki] * (8 * W + 38);
    work = std::max(work, smp.cap[ki] * 12 + smp.claimed[ki] * (20 + 16 * W));
  }
  return rows + work + (8ull << 20);
}

static int run_finalize(kh_server* S, SampleState& smp, kh_table** outs,
                        bool others_resident) {
  kh_ctx* ctx = S->ctx;
  hipStream_t s = S->stream;
  if (smp.error != KH_OK) return fail(smp.error, "%s", smp.error_msg.c_str());
  for (int ki = 0; ki < S->nk; ++ki) outs[ki] = nullptr;
  if (others_resident) {  // refuse before touching the tables if it may not fit
    Pool& pool = ctx->pool;
    std::lock_guard<std::recursive_mutex> lk(pool.mu);
    const uint64_t in_use = pool.held - pool.cached_bytes;
    const uint64_t need = finalize_bytes(S, smp);
    if (pool.budget && in_use + need > pool.budget) {
      fail(KH_ENOMEM, "finalize may need %llu bytes; %llu of the %llu-byte budget are in "
                      "use: finalize other samples or free tables first",
           (unsigned long long)need, (unsigned long long)in_use,
           (unsigned long long)pool.budget);
      return kNoRoom;
    }
  }
  for (int ki = 0; ki < S->nk; ++ki) {
    kh_params p = S->params;
    p.k = S->ks[ki];
    kh_table* t = nullptr;
    int rc = make_table(ctx, p.k, &t);
    if (rc == KH_OK) {
      t->n_windows = smp.windows[ki];
      if (smp.cap[ki] == 0) {  // no bases: an empty table
        rc = KH_OK;
      } else {
        RecountFn recount = [&](HeavyEntry* heavy, uint32_t* index, uint32_t mask) -> int {
          std::vector<TileDesc> descs;
          Arena& ar = smp.arena;
          for (auto& c : ar.chunks)
            for (int64_t p0 = c.first; p0 < c.second; p0 += kTile) {
              TileDesc d{};
              d.bases = ar.bases.p;
              d.hq = ar.hq.p;
              d.bad = ar.bad.p;
              d.st = ar.st.p;
              d.base_words = ar.cap / 32 + 4;
              d.plane_words = ar.cap / 64 + 4;
              d.p0 = p0;
              d.hi = c.second;
              d.table = smp.table[ki].p;
              d.capacity = smp.cap[ki];
              d.heavy = heavy;
              d.heavy_index = index;
              d.heavy_mask = mask;
              descs.push_back(d);
            }
          if (descs.empty()) return KH_OK;
          Buf<TileDesc> dd(&ctx->pool);
          KH_TRY(dd.alloc(descs.size()));
          HIP_TRY(hipMemcpyAsync(dd.p, descs.data(), descs.size() * sizeof(TileDesc),
                                 hipMemcpyHostToDevice, s));
          WindowArgs wa{};
          wa.k = p.k;
          wa.ctr = ctx->ctr;
          wa.tiles = dd.p;
          wa.n_tiles = (int64_t)descs.size();
          launch_windows(wa, 3, s);
          HIP_TRY(hipGetLastError());
          HIP_TRY(hipStreamSynchronize(s));
          return KH_OK;
        };
        rc = finish_rows(ctx, ctx->ctr, smp.table[ki].p, smp.cap[ki], p, recount, s, t);
      }
    }
    if (rc != KH_OK) {
      if (t) kh_table_free(t);
      for (int j = 0; j < ki; ++j) {
        kh_table_free(outs[j]);
        outs[j] = nullptr;
      }
      return rc;
    }
    outs[ki] = t;
  }
  return KH_OK;
}

// ----------------------------------------------------------------- worker --

// Device bytes a request is expected to need: its bases packed (5/8 B),
// and for each k the table its sample will grow to (as table_reserve plans
// it: keys held plus its windows at the sample's rate of new keys so far,
// 0.3 for a new sample, at load 0.5, power-of-two sizes), counted in full
// while the table is larger than now since a rehash holds old and new.
static uint64_t request_bytes(kh_server* S, const Request* r) {
  const int64_t nb = r->reads.n_reads > 0 ? r->reads.offsets[r->reads.n_reads] : 0;
  double b = 5.0 / 8.0 * (double)nb;
  auto it = S->samples.find(r->sample);
  const SampleState* smp = it != S->samples.end() ? it->second.get() : nullptr;
  for (int ki = 0; ki < S->nk; ++ki) {
    const uint64_t cap = smp ? smp->cap[ki] : 0;
    const uint64_t claimed = smp ? smp->claimed[ki] : 0;
    const uint64_t windows = smp ? smp->windows[ki] : 0;
    const double rate = windows ? std::max(0.02, (double)claimed / (double)windows) : 0.3;
    const double expect = (double)claimed + rate * (double)nb;
    const uint64_t need =
        pow2_at_least(std::max<uint64_t>(1u << 20, (uint64_t)(expect / 0.5)));
    if (need > cap) b += (double)need * (double)slot_layout(table_chunks(S->ks[ki])).stride;
  }
  return (uint64_t)b;
}

// Does a sample other than `sample` hold device memory?
static bool others_hold_memory(kh_server* S, uint64_t sample) {
  for (auto& kv : S->samples)
    if (kv.first != sample && (kv.second->arena.cap > 0 || kv.second->cap[0] > 0)) return true;
  return false;
}

// Admit a request needing `want` more bytes?  Device memory in use (the
// pool's blocks minus those free for reuse) plus the reserves of admitted
// requests must stay under 60 % of the budget (the rest is room for
// finalizing samples and for rehash transients).
static bool memory_ok(kh_server* S, uint64_t want) {
  Pool& pool = S->ctx->pool;
  std::lock_guard<std::recursive_mutex> lk(pool.mu);  // tables are freed by callers
  const uint64_t in_use = pool.held - pool.cached_bytes;
  return pool.budget == 0 ||
         (double)(in_use + S->reserved + want) < 0.6 * (double)pool.budget;
}

// Book a launch's result on its requests (under the lock): a request is done
// once all of its chunks have been counted.
static void complete_takes(kh_server* S, std::vector<Take>& takes, int rc,
                           Clock::time_point t_end) {
  for (Take& t : takes) {
    if (rc != KH_OK && t.smp->error == KH_OK) {
      t.smp->error = rc;
      t.smp->error_msg = kh_last_error();
    }
    Request* r = t.r;
    if (--r->inflight == 0 && r->next >= r->reads.n_reads && !r->done) {
      r->done = true;
      r->status = rc == KH_OK ? t.smp->error : rc;
      if (r->status != KH_OK) r->msg = t.smp->error_msg;
      r->t_done = t_end;
      S->reserved -= r->reserve;
      r->reserve = 0;
      t.smp->open_requests--;
      S->n_done++;
      S->active.erase(std::find(S->active.begin(), S->active.end(), r));
    }
  }
  S->cv_done.notify_all();
}

static void finish_and_book(kh_server* S, std::unique_ptr<Launch>& L) {
  const auto t0 = Clock::now();
  const int rc = finish_launch(S, *L);
  const auto t1 = Clock::now();
  std::lock_guard<std::mutex> lk(S->mu);
  S->busy_s += std::chrono::duration<double>(t1 - t0).count();
  complete_takes(S, L->takes, rc, t1);
  L.reset();
}

static void worker_main(kh_server* S) {
  (void)hipSetDevice(S->ctx->device);
  std::unique_ptr<Launch> prev;  // enqueued, not yet finished
  for (;;) {
    std::vector<Take> takes;
    std::vector<FinalizeCmd*> fins;
    bool stopping = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (!prev)
        S->cv_work.wait(lk, [&] {
          return S->stop || !S->pending.empty() || !S->active.empty() ||
                 !S->finalize_q.empty();
        });
      stopping = S->stop;
      if (!stopping) {
        for (auto it = S->finalize_q.begin(); it != S->finalize_q.end();) {
          auto sm = S->samples.find((*it)->sample);
          if (sm == S->samples.end() || sm->second->open_requests == 0) {
            fins.push_back(*it);
            it = S->finalize_q.erase(it);
          } else {
            ++it;
          }
        }
        // admission, in arrival order: a free slot and room in the HBM
        // budget (or, so that work never stalls, the oldest request when
        // nothing runs and no other sample holds device memory; samples that
        // are complete but not finalized hold theirs until the client
        // finalizes)
        while (!S->pending.empty() && (int)S->active.size() < (int)S->cfg.max_active) {
          Request* r = S->pending.front();
          const uint64_t want = request_bytes(S, r);
          if (!memory_ok(S, want) && !(S->active.empty() && !others_hold_memory(S, r->sample)))
            break;
          S->pending.pop_front();
          r->reserve = want;
          const int64_t nb = r->reads.n_reads > 0 ? r->reads.offsets[r->reads.n_reads] : 0;
          r->reserve_per_base = (double)want / (double)std::max<int64_t>(1, nb);
          S->reserved += want;
          S->active.push_back(r);
        }
        S->max_active_seen = std::max<uint64_t>(S->max_active_seen, S->active.size());
        // build one launch: chunks of the admitted requests, round robin (the
        // oldest request alone after a launch that did not fit)
        const bool solo = S->solo_next;
        S->solo_next = false;
        int64_t bases = 0;
        bool progress = true;
        while (progress && bases < S->cfg.batch_bases) {
          progress = false;
          for (Request* r : S->active) {
            if (r->next >= r->reads.n_reads) continue;
            const int64_t r1 = std::min<int64_t>(r->reads.n_reads, r->next + S->cfg.chunk_reads);
            const int64_t nb = r->reads.offsets[r1] - r->reads.offsets[r->next];
            if (!takes.empty() && bases + nb > S->cfg.batch_bases) continue;
            Take t{};
            t.r = r;
            t.smp = S->samples[r->sample].get();
            t.r0 = r->next;
            t.r1 = r1;
            t.reserve =
                std::min<uint64_t>(r->reserve, (uint64_t)((double)nb * r->reserve_per_base));
            r->reserve -= t.reserve;
            S->reserved -= t.reserve;
            takes.push_back(t);
            r->next = r1;
            r->inflight++;
            bases += nb;
            progress = true;
            if (S->cfg.plain || solo || bases >= S->cfg.batch_bases) break;
          }
          if (S->cfg.plain || solo) break;
        }
      }
    }
    if (stopping) {  // the launch in flight finishes; queued ones fail later
      if (prev) finish_and_book(S, prev);
      break;
    }
    // ---- device work, outside the lock
    for (FinalizeCmd* f : fins) {
      std::unique_ptr<SampleState> smp;
      bool others = false;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        auto sm = S->samples.find(f->sample);
        if (sm != S->samples.end()) {
          smp = std::move(sm->second);
          S->samples.erase(sm);
        }
        others = !S->samples.empty();
      }
      int rc = smp ? run_finalize(S, *smp, f->outs, others)
                   : fail(KH_ENOTFOUND, "unknown sample %llu",
                          (unsigned long long)f->sample);
      std::string msg = rc == KH_OK ? std::string() : std::string(kh_last_error());
      if (rc == kNoRoom) {  // nothing was touched: the sample stays resident
        rc = KH_ENOMEM;
        std::lock_guard<std::mutex> lk(S->mu);
        S->samples[f->sample] = std::move(smp);
      }
      smp.reset();  // arena and tables return to the pool
      std::lock_guard<std::mutex> lk(S->mu);
      f->status = rc;
      f->msg = msg;
      f->done = true;
      S->cv_done.notify_all();
    }
    std::unique_ptr<Launch> cur;
    if (!takes.empty()) {
      cur = std::make_unique<Launch>(&S->ctx->pool);
      cur->takes = std::move(takes);
      const auto t0 = Clock::now();
      int rc = stage_launch(S, *cur);
      if (rc == KH_OK) rc = enqueue_launch(S, *cur);
      const auto t1 = Clock::now();
      std::lock_guard<std::mutex> lk(S->mu);
      S->busy_s += std::chrono::duration<double>(t1 - t0).count();
      if (rc == kNoRoom) {
        bool several = false;
        for (const Take& t : cur->takes) several = several || t.r != cur->takes[0].r;
        if (several) {  // nothing was counted: hand the chunks back, retry smaller
          for (const Take& t : cur->takes) {
            t.r->next = std::min(t.r->next, t.r0);
            t.r->inflight--;
            t.r->reserve += t.reserve;
            S->reserved += t.reserve;
          }
          S->solo_next = true;
          ++S->n_retried;
          cur.reset();
        } else {
          rc = KH_ENOMEM;  // one request alone does not fit the budget
        }
      }
      if (cur && rc != KH_OK) {
        complete_takes(S, cur->takes, rc, t1);
        cur.reset();
      }
    }
    if (prev) finish_and_book(S, prev);
    if (cur && S->cfg.plain) finish_and_book(S, cur);  // plain: stop and wait
    prev = std::move(cur);
    {  // requests without reads complete at once
      std::lock_guard<std::mutex> lk(S->mu);
      for (size_t i = 0; i < S->active.size();) {
        Request* r = S->active[i];
        if (!r->done && r->reads.n_reads == 0 && r->inflight == 0) {
          r->done = true;
          r->t_done = Clock::now();
          S->reserved -= r->reserve;
          r->reserve = 0;
          S->samples[r->sample]->open_requests--;
          S->n_done++;
          S->active.erase(S->active.begin() + i);
          S->cv_done.notify_all();
        } else {
          ++i;
        }
      }
    }
  }
}

// -------------------------------------------------------------------- API --

static void release_streams(kh_server* S) {
  if (S->stream) (void)hipStreamDestroy(S->stream);
  if (S->copy) (void)hipStreamDestroy(S->copy);
  for (int i = 0; i < 2; ++i) {
    if (S->copy_ev[i]) (void)hipEventDestroy(S->copy_ev[i]);
    if (S->done_ev[i]) (void)hipEventDestroy(S->done_ev[i]);
  }
}

extern "C" void kh_server_default_config(kh_server_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->max_active = 16;
  c->queue_cap = 1024;
  c->chunk_reads = 16384;
  c->batch_bases = 32ll << 20;
  c->plain = 0;
}

extern "C" int kh_server_create(kh_server** out, int device, uint64_t hbm_budget_bytes,
                                const kh_params* params, const uint32_t* ks, int nk,
                                const kh_server_config* cfg) {
  if (!out || !ks) return fail(KH_EINVAL, "NULL argument");
  *out = nullptr;
  if (nk < 1 || nk > kMaxK) return fail(KH_EINVAL, "nk must be in 1..%d", (int)kMaxK);
  KH_TRY(check_params(params));
  if (params->use_bloom)
    return fail(KH_EINVAL, "serving counts exactly across batches: use_bloom must be 0");
  if (params->owner_shards > 1)
    return fail(KH_EINVAL, "serving keeps whole tables: owner_shards must be 0 or 1");
  for (int i = 0; i < nk; ++i) {
    kh_params q = *params;
    q.k = ks[i];
    KH_TRY(check_params(&q));
  }
  kh_server_config c;
  kh_server_default_config(&c);
  if (cfg) c = *cfg;
  if (c.plain) c.max_active = 1;
  if (c.max_active < 1 || c.queue_cap < 1 || c.chunk_reads < 1 || c.batch_bases < 1)
    return fail(KH_EINVAL, "bad server configuration");
  kh_ctx* ctx = nullptr;
  KH_TRY(kh_create(&ctx, device, hbm_budget_bytes, nullptr, nullptr, nullptr));
  if (hbm_budget_bytes == 0) {  // admission needs a budget: 85 % of the device
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
      ctx->pool.budget = (uint64_t)(0.85 * (double)total_b);
    else
      (void)hipGetLastError();
  }
  kh_server* S = new (std::nothrow) kh_server();
  if (!S) {
    kh_destroy(ctx);
    return fail(KH_ENOMEM, "host allocation failed");
  }
  S->ctx = ctx;
  S->params = *params;
  S->nk = nk;
  for (int i = 0; i < nk; ++i) S->ks[i] = ks[i];
  S->cfg = c;
  // Test hook: tables start this small and grow only when a launch fills
  // them, which exercises the overflow replay.
  if (const char* f = std::getenv("KMERHIP_SERVER_TABLE_SLOTS"))
    S->force_slots = std::max<uint64_t>(64, std::strtoull(f, nullptr, 10));
  bool ok = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&S->copy, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < 2; ++i)
    ok = hipEventCreateWithFlags(&S->copy_ev[i], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&S->done_ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    release_streams(S);
    kh_destroy(ctx);
    delete S;
    return fail(KH_EDEVICE, "stream or event creation failed");
  }
  for (auto& st : S->stage) st = std::make_unique<StageSet>(&ctx->pool);
  S->worker = std::thread(worker_main, S);
  *out = S;
  return KH_OK;
}

extern "C" int kh_server_submit(kh_server* S, uint64_t sample, const kh_reads* reads,
                                uint64_t* ticket) {
  if (!S || !reads || !ticket) return fail(KH_EINVAL, "NULL argument");
  if (reads->on_device) return fail(KH_EINVAL, "serving takes host reads");
  if (reads->n_reads < 0) return fail(KH_EINVAL, "n_reads < 0");
  if (reads->n_reads > 0) {
    if (!reads->offsets || !reads->seq || !reads->qual) return fail(KH_EINVAL, "NULL read array");
    if (reads->offsets[0] != 0) return fail(KH_EINVAL, "offsets[0] must be 0");
    for (int64_t i = 0; i < reads->n_reads; ++i)
      if (reads->offsets[i + 1] < reads->offsets[i])
        return fail(KH_EINVAL, "offsets decrease at read %lld", (long long)i);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->pending.size() >= S->cfg.queue_cap)
    return fail(KH_EAGAIN, "request queue is full (%u waiting)", S->cfg.queue_cap);
  auto r = std::make_unique<Request>();
  r->ticket = S->next_ticket++;
  r->sample = sample;
  r->reads = *reads;
  r->t_submit = Clock::now();
  auto& smp = S->samples[sample];
  if (!smp) smp = std::make_unique<SampleState>(&S->ctx->pool, sample);
  smp->open_requests++;
  S->pending.push_back(r.get());
  *ticket = r->ticket;
  S->requests[r->ticket] = std::move(r);
  S->cv_work.notify_all();
  return KH_OK;
}

static int ticket_state(kh_server* S, uint64_t ticket, int* done, double* latency_ms) {
  auto it = S->requests.find(ticket);
  if (it == S->requests.end()) return fail(KH_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second.get();
  if (done) *done = r->done ? 1 : 0;
  if (latency_ms)
    *latency_ms = r->done ? std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count()
                          : -1.0;
  if (r->done && r->status != KH_OK)
    return fail(r->status, "batch %llu failed: %s", (unsigned long long)ticket, r->msg.c_str());
  return KH_OK;
}

extern "C" int kh_server_poll(kh_server* S, uint64_t ticket, int* done, double* latency_ms) {
  if (!S) return fail(KH_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  return ticket_state(S, ticket, done, latency_ms);
}

extern "C" int kh_server_wait(kh_server* S, uint64_t ticket, double* latency_ms) {
  if (!S) return fail(KH_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->requests.find(ticket);
  if (it == S->requests.end()) return fail(KH_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second.get();
  S->cv_done.wait(lk, [&] { return r->done; });
  return ticket_state(S, ticket, nullptr, latency_ms);
}

extern "C" int kh_server_finalize(kh_server* S, uint64_t sample, kh_table** outs) {
  if (!S || !outs) return fail(KH_EINVAL, "NULL argument");
  FinalizeCmd cmd;
  cmd.sample = sample;
  cmd.outs = outs;
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->samples.find(sample) == S->samples.end())
    return fail(KH_ENOTFOUND, "unknown sample %llu", (unsigned long long)sample);
  S->finalize_q.push_back(&cmd);
  S->cv_work.notify_all();
  S->cv_done.wait(lk, [&] { return cmd.done; });
  if (cmd.status != KH_OK) return fail(cmd.status, "%s", cmd.msg.c_str());
  return KH_OK;
}

extern "C" int kh_server_stats(kh_server* S, double out[17]) {
  if (!S || !out) return fail(KH_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  out[0] = (double)S->n_done;
  out[1] = (double)S->n_launches;
  out[2] = S->windows_total;
  out[3] = S->busy_s;
  out[4] = (double)S->max_active_seen;
  out[5] = (double)S->samples.size();
  {
    std::lock_guard<std::recursive_mutex> plk(S->ctx->pool.mu);
    out[6] = (double)S->ctx->pool.held;
    out[15] = (double)(S->ctx->pool.held - S->ctx->pool.cached_bytes);
  }
  out[16] = (double)S->reserved;
  out[7] = (double)S->n_rehash;
  out[8] = (double)S->n_replayed;
  out[9] = S->pack_s;
  out[10] = S->grow_s;
  out[11] = (double)S->ctx->pool.peak;
  out[12] = (double)S->ctx->pool.n_alloc;
  out[13] = S->ctx->pool.alloc_s;
  out[14] = (double)S->n_retried;
  return KH_OK;
}

extern "C" int kh_server_destroy(kh_server* S) {
  if (!S) return fail(KH_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (FinalizeCmd* f : S->finalize_q) {  // callers blocked in finalize
      f->status = KH_EAGAIN;
      f->msg = "server destroyed";
      f->done = true;
    }
    S->finalize_q.clear();
    for (auto& kv : S->requests)
      if (!kv.second->done) {
        kv.second->done = true;
        kv.second->status = KH_EAGAIN;
      }
    S->cv_done.notify_all();
  }
  S->samples.clear();
  (void)hipDeviceSynchronize();
  for (auto& st : S->stage)
    if (st) {
      for (PinnedBuf* b : {&st->hoff, &st->hdesc, &st->hctr})
        if (b->p) (void)hipHostFree(b->p);
      st.reset();
    }
  release_streams(S);
  kh_destroy(S->ctx);
  delete S;
  return KH_OK;
}
