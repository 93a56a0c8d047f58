// De Bruijn graph traversal on the device (paper Section II-C): the kept
// k-mers of a table are the vertices, each with its two-letter extension
// code, and a contig is a maximal path of k-mers joined by unique
// high-quality extensions.
//
// Definition (the same as the contig oracle's):
//  * k-mer S joins S' = S[1..k) + b when S's right code is b, S' is a kept
//    k-mer and S''s left code is S[0] (the edge is mutual); codes of a k-mer
//    read on its reverse strand swap sides and complement; an edge from a
//    k-mer to itself or to its reverse complement is dropped;
//  * every k-mer is in exactly one contig, a maximal path or a cycle;
//  * a path is written in the orientation that is lexicographically smaller
//    than its reverse complement; a cycle is opened at its smallest k-mer in
//    canonical orientation and written walking right (k + n - 1 bases);
//  * contigs are listed by their smallest k-mer, with their number of
//    k-mers and the sum of their counts.
//
// Method.  A k-mer read in orientation o (0 canonical, 1 reverse
// complement) and walked to the right is a *state* 2i + o.  Every state has
// at most one successor, so the states form 2 directed chains per path
// (one per reading direction) and 2 directed cycles per cycle.  After an
// open-addressing index over the sorted rows (row -> slot) gives each state
// its successor, pointer jumping (Wyllie's list ranking, log2 rounds) gives
// every state its chain's end, its distance to it and the smallest k-mer
// behind it.  States still moving after enough rounds to cover any path lie
// on cycles: each cycle is cut in front of its smallest k-mer's canonical
// state, and the ranking is repeated.  A k-mer then knows both chains that
// run through it, picks the one the contig is written in, its position in
// it and its contig (numbered by smallest k-mer with a prefix sum), and
// writes its own bases.
#include <algorithm>
#include <cstring>
#include <vector>

#include "kh_device.hpp"
#include "kh_host.hpp"
#include "kh_rows.hpp"

using namespace kh;

namespace {

constexpr int kTB = 256;

__device__ __forceinline__ uint64_t row_hash(const uint64_t* w, int W) {
  uint64_t h = 0x243f6a8885a308d3ull;
  for (int j = 0; j < W; ++j) h = fmix64(h ^ w[j]);
  return h;
}

__device__ __forceinline__ int base_of(uint8_t c) {
  switch (c) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
  }
}

__device__ __forceinline__ uint8_t comp_code(uint8_t c) {
  switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    default: return c;
  }
}

template <int W>
__device__ __forceinline__ void load_row(const uint64_t* keys, int64_t i, uint64_t (&w)[W]) {
#pragma unroll
  for (int j = 0; j < W; ++j) w[j] = keys[i * W + j];
}

template <int W>
__device__ __forceinline__ bool same_key(const uint64_t* keys, int64_t r, const uint64_t (&q)[W]) {
  bool eq = true;
#pragma unroll
  for (int j = 0; j < W; ++j) eq = eq && keys[r * W + j] == q[j];
  return eq;
}

template <int W>
__global__ __launch_bounds__(kTB) void k_index_build(const uint64_t* keys, int64_t n,
                                                     uint32_t* slots, uint64_t mask) {
  const int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (i >= n) return;
  uint64_t w[W];
  load_row<W>(keys, i, w);
  uint64_t x = row_hash(w, W) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {  // capacity > n: ends
    if (atomicCAS(&slots[x], 0u, (uint32_t)(i + 1)) == 0u) return;
    x = (x + 1) & mask;
  }
}

template <int W>
__device__ __forceinline__ int64_t find_row(const uint64_t* keys, const uint32_t* slots,
                                            uint64_t mask, const uint64_t (&q)[W]) {
  uint64_t x = row_hash(q, W) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const uint32_t v = slots[x];
    if (v == 0u) return -1;
    if (same_key<W>(keys, (int64_t)v - 1, q)) return (int64_t)v - 1;
    x = (x + 1) & mask;
  }
  return -1;
}

// Successor of both states of every k-mer (-1: the chain ends).
template <int W>
__global__ __launch_bounds__(kTB) void k_link(const uint64_t* keys, const uint8_t* codes,
                                              int64_t n, uint32_t k, const uint32_t* slots,
                                              uint64_t mask, int64_t* succ) {
  const int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (i >= n) return;
  const int top = 2 * (int)k - 64 * (W - 1);
  uint64_t s[W];
  load_row<W>(keys, i, s);
  const int first = (int)((s[0] >> (top - 2)) & 3), last = (int)(s[W - 1] & 3);
  const uint8_t letters[4] = {'A', 'C', 'G', 'T'};
  // state 2i: canonical reading, step right
  int64_t nx = -1;
  int b = base_of(codes[2 * i + 1]);
  if (b >= 0) {
    uint64_t t[W], r[W];
    push_right<W>(s, b, top, t);
    revcomp_words<W>(t, k, r);
    const bool fwd = !words_less<W>(r, t);
#pragma unroll
    for (int j = 0; j < W; ++j) r[j] = fwd ? t[j] : r[j];
    const int64_t j = find_row<W>(keys, slots, mask, r);
    if (j >= 0 && j != i) {
      const uint8_t back = fwd ? codes[2 * j] : comp_code(codes[2 * j + 1]);
      if (back == letters[first]) nx = 2 * j + (fwd ? 0 : 1);
    }
  }
  succ[2 * i] = nx;
  // state 2i + 1: reverse-complement reading, step right = canonical step left
  nx = -1;
  b = base_of(codes[2 * i]);
  if (b >= 0) {
    uint64_t t[W], r[W];
    push_left<W>(s, b, top, t);
    revcomp_words<W>(t, k, r);
    const bool fwd = !words_less<W>(r, t);
#pragma unroll
    for (int j = 0; j < W; ++j) r[j] = fwd ? t[j] : r[j];
    const int64_t j = find_row<W>(keys, slots, mask, r);
    if (j >= 0 && j != i) {
      const uint8_t back = fwd ? codes[2 * j + 1] : comp_code(codes[2 * j]);
      if (back == letters[last]) nx = 2 * j + (fwd ? 1 : 0);
    }
  }
  succ[2 * i + 1] = nx;
}

// Pointer-jumping record of a state, one 32-byte line segment, so that a
// jump reads the record it points at in one access.
struct alignas(32) Rec {
  int64_t nxt;   // state reached so far (-1: the chain's end is behind)
  int64_t last;  // last state of the chain reached so far
  int64_t dist;  // states from here to `last`
  uint32_t mn;   // smallest k-mer from here to `last` (inclusive)
  uint32_t pad;
};

// Raise *moving if any state of the block is still moving (a plain store of
// 1 per block; only "any" is needed, so no counting atomics).
__device__ __forceinline__ void flag_moving(unsigned int* moving, bool on) {
  if (__syncthreads_or(on) && threadIdx.x == 0) *moving = 1u;
}

__global__ __launch_bounds__(kTB) void k_jump_init(const int64_t* succ, int64_t m, Rec* a,
                                                   unsigned int* moving) {
  const int64_t s = (int64_t)blockIdx.x * kTB + threadIdx.x;
  const bool in = s < m;
  const int64_t t = in ? succ[s] : -1;
  if (in) {
    Rec r;
    r.nxt = t;
    r.last = t >= 0 ? t : s;
    r.dist = t >= 0 ? 1 : 0;
    r.mn = (uint32_t)(s >> 1);
    r.pad = 0;
    a[s] = r;
  }
  flag_moving(moving, in && t >= 0);
}

// One doubling round: a state's segment [s, nxt) absorbs the segment of
// the state it points at.
__global__ __launch_bounds__(kTB) void k_jump(const Rec* a, Rec* b, int64_t m,
                                              unsigned int* moving) {
  const int64_t s = (int64_t)blockIdx.x * kTB + threadIdx.x;
  bool on = false;
  if (s < m) {
    Rec r = a[s];
    if (r.nxt >= 0) {
      const Rec u = a[r.nxt];
      r.nxt = u.nxt;
      r.last = u.last;
      r.dist += u.dist;
      r.mn = min(r.mn, u.mn);
      on = r.nxt >= 0;
    }
    b[s] = r;
  }
  flag_moving(moving, on);
}

// States still moving lie on cycles (every path has ended): open each cycle
// in front of the canonical state of its smallest k-mer, and end its
// reverse reading at that k-mer's other state.
__global__ __launch_bounds__(kTB) void k_cut_cycles(const Rec* a, int64_t m, int64_t* succ,
                                                    uint8_t* on_cycle) {
  const int64_t s = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (s >= m || a[s].nxt < 0) return;
  const int64_t c = 2 * (int64_t)a[s].mn;  // mn covers the whole cycle
  if (succ[s] == c || s == c + 1) succ[s] = -1;
  on_cycle[s >> 1] = 1;
}

// Per k-mer: the chain its contig is written in, its place there, and (at
// the contig's smallest k-mer) the contig's length.
template <int W>
__global__ __launch_bounds__(kTB) void k_resolve(const uint64_t* keys, int64_t n, uint32_t k,
                                                 const Rec* a, const uint8_t* on_cycle,
                                                 int64_t* start_of, int64_t* pos_of,
                                                 uint64_t* rep_flag, uint64_t* rep_len,
                                                 unsigned int* bad) {
  const int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (i >= n) return;
  const int64_t sA = a[2 * i + 1].last ^ 1;  // start of the chain through 2i
  const int64_t sB = a[2 * i].last ^ 1;      // start of the chain through 2i+1
  bool useA;
  if (on_cycle[i]) {
    useA = sA == 2 * (int64_t)a[sA].mn;  // opened at the canonical state
  } else {  // the smaller first k-mer decides which reading is smaller
    uint64_t x[W], y[W], r[W];
    load_row<W>(keys, sA >> 1, x);
    if (sA & 1) {
      revcomp_words<W>(x, k, r);
#pragma unroll
      for (int j = 0; j < W; ++j) x[j] = r[j];
    }
    load_row<W>(keys, sB >> 1, y);
    if (sB & 1) {
      revcomp_words<W>(y, k, r);
#pragma unroll
      for (int j = 0; j < W; ++j) y[j] = r[j];
    }
    useA = !words_less<W>(y, x);
  }
  const int64_t start = useA ? sA : sB;
  const int64_t me = useA ? 2 * i : 2 * i + 1;
  const int64_t pos = a[start].dist - a[me].dist;
  if (pos < 0) atomicOr(bad, 1u);  // chains not symmetric: refuse to place
  start_of[i] = start;
  pos_of[i] = 2 * (pos < 0 ? 0 : pos) + (me & 1);  // place, reading
  const bool rep = (int64_t)a[start].mn == i;
  rep_flag[i] = rep ? 1 : 0;
  rep_len[i] = rep ? (uint64_t)k + (uint64_t)a[start].dist : 0;
}

// Contig lengths in contig order (representatives are in k-mer order).
__global__ __launch_bounds__(kTB) void k_contig_lens(const uint64_t* rep_flag,
                                                     const uint64_t* cidx,
                                                     const uint64_t* rep_len, int64_t n,
                                                     uint64_t* lens) {
  const int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (i >= n || !rep_flag[i]) return;
  lens[cidx[i]] = rep_len[i];
}

template <int W>
__global__ __launch_bounds__(kTB) void k_emit(const uint64_t* keys, const uint32_t* counts,
                                              int64_t n, uint32_t k, const Rec* a,
                                              const uint8_t* on_cycle, const int64_t* start_of,
                                              const int64_t* pos_of, const uint64_t* cidx,
                                              const uint64_t* offs, uint64_t n_contigs,
                                              char* seq, int64_t* n_kmers,
                                              unsigned long long* depth, uint8_t* cycle,
                                              uint32_t* row_contig, unsigned int* bad) {
  const int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (i >= n) return;
  const int64_t start = start_of[i], pos = pos_of[i] >> 1;
  const uint64_t c = cidx[a[start].mn];
  if (c >= n_contigs) {  // not a numbered contig: inconsistent chains
    atomicOr(bad, 2u);
    return;
  }
  const int64_t base = (int64_t)offs[c];
  if (pos + (int64_t)k > (int64_t)(offs[c + 1] - offs[c])) {  // outside its contig
    atomicOr(bad, 4u);
    return;
  }
  row_contig[i] = (uint32_t)c;
  uint64_t w[W], r[W];
  load_row<W>(keys, i, w);
  if (pos_of[i] & 1) {  // read on the reverse strand in this contig
    revcomp_words<W>(w, k, r);
#pragma unroll
    for (int j = 0; j < W; ++j) w[j] = r[j];
  }
  const char letters[4] = {'A', 'C', 'G', 'T'};
  if (pos == 0) {
    for (uint32_t p = 0; p < k; ++p) {  // base p of the k-mer
      const int bit = 2 * (int)(k - 1 - p);
      const int wi = W - 1 - bit / 64;
      seq[base + p] = letters[(w[wi] >> (bit % 64)) & 3];
    }
    n_kmers[c] = a[start].dist + 1;
    cycle[c] = on_cycle[i];
  } else {
    seq[base + (int64_t)k - 1 + pos] = letters[w[W - 1] & 3];
  }
  atomicAdd(&depth[c], (unsigned long long)counts[i]);
}

// ---- exclusive prefix sum over uint64 (block scan + recursion on block sums)

constexpr int kScanItems = 4;
constexpr int kScanTile = kTB * kScanItems;

__global__ __launch_bounds__(kTB) void k_scan_tile(const uint64_t* in, uint64_t* out,
                                                   int64_t n, uint64_t* sums) {
  __shared__ uint64_t wsum[kTB / 64];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems], run = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (t0 + j < n) ? in[t0 + j] : 0;
    run += v[j];
  }
  unsigned long long inc = run;  // inclusive scan of the thread totals in the wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint64_t before = inc - run;
  for (int q = 0; q < wave; ++q) before += wsum[q];
  uint64_t acc = before;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (t0 + j < n) out[t0 + j] = acc;
    acc += v[j];
  }
  if (threadIdx.x == kTB - 1) sums[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kTB) void k_scan_add(uint64_t* out, int64_t n,
                                                  const uint64_t* offs) {
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  const uint64_t add = offs[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (t0 + j < n) out[t0 + j] += add;
}

// out[i] = in[0] + ... + in[i-1]; *total (device) = the sum of all.
int scan_exclusive(Pool* pool, const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total,
                   hipStream_t s) {
  const int64_t blocks = (n + kScanTile - 1) / kScanTile;
  if (n == 0) {
    launch_fill_u64(total, 1, 0ull, s);
    return KH_OK;
  }
  Buf<uint64_t> sums(pool), offs(pool);
  KH_TRY(sums.alloc(blocks));
  KH_TRY(offs.alloc(blocks));
  hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)blocks), dim3(kTB), 0, s, in, out, n, sums.p);
  HIP_TRY(hipGetLastError());
  if (blocks == 1) {
    HIP_TRY(hipMemcpyAsync(total, sums.p, 8, hipMemcpyDeviceToDevice, s));
    launch_fill_u64(offs.p, 1, 0ull, s);
  } else {
    KH_TRY(scan_exclusive(pool, sums.p, offs.p, blocks, total, s));
  }
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)blocks), dim3(kTB), 0, s, out, n, offs.p);
  HIP_TRY(hipGetLastError());
  return KH_OK;
}

unsigned grid(int64_t n) { return (unsigned)((n + kTB - 1) / kTB); }

template <int W>
int traverse_w(kh_ctx* ctx, const kh_table* t, hipStream_t s, kh_contigs* out) {
  Pool* pool = &ctx->pool;
  const int64_t n = t->n_rows;
  const uint32_t k = t->k;
  const int64_t m = 2 * n;
  // ---- index: canonical key -> row
  uint64_t cap = 1024;
  while (cap < (uint64_t)(2 * n)) cap <<= 1;
  Buf<uint32_t> slots(pool);
  KH_TRY(slots.alloc(cap));
  launch_fill_u64(reinterpret_cast<uint64_t*>(slots.p), cap / 2, 0ull, s);
  hipLaunchKernelGGL((k_index_build<W>), dim3(grid(n)), dim3(kTB), 0, s, t->keys, n, slots.p,
                     cap - 1);
  HIP_TRY(hipGetLastError());
  // ---- successors of every state
  Buf<int64_t> succ(pool);
  KH_TRY(succ.alloc(m));
  hipLaunchKernelGGL((k_link<W>), dim3(grid(n)), dim3(kTB), 0, s, t->keys, t->codes, n, k,
                     slots.p, cap - 1, succ.p);
  HIP_TRY(hipGetLastError());
  slots.reset();
  // ---- list ranking by pointer jumping
  Buf<Rec> recs[2] = {Buf<Rec>(pool), Buf<Rec>(pool)};
  KH_TRY(recs[0].alloc(m));
  KH_TRY(recs[1].alloc(m));
  Buf<uint8_t> on_cycle(pool);
  KH_TRY(on_cycle.alloc(n + 8));
  launch_fill_u64(reinterpret_cast<uint64_t*>(on_cycle.p), (n + 7) / 8, 0ull, s);
  Buf<uint64_t> mv(pool);
  KH_TRY(mv.alloc(1));
  unsigned int* moving = reinterpret_cast<unsigned int*>(mv.p);
  int max_rounds = 2;  // 2^(rounds - 2) >= states: every path has ended by then
  while ((1ll << (max_rounds - 2)) < m) ++max_rounds;
  int cur = 0;
  unsigned int on = 0;
  // Rank the chains of `succ`; the result is left in recs[cur] and `on`
  // tells whether states are still moving (those on cycles).
  auto rank = [&]() -> int {
    launch_fill_u64(mv.p, 1, 0ull, s);
    hipLaunchKernelGGL(k_jump_init, dim3(grid(m)), dim3(kTB), 0, s, succ.p, m, recs[0].p,
                       moving);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&on, moving, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    cur = 0;
    for (int r = 0; r < max_rounds && on; ++r) {
      launch_fill_u64(mv.p, 1, 0ull, s);
      hipLaunchKernelGGL(k_jump, dim3(grid(m)), dim3(kTB), 0, s, recs[cur].p, recs[cur ^ 1].p,
                         m, moving);
      HIP_TRY(hipGetLastError());
      cur ^= 1;
      ++out->rounds;
      HIP_TRY(hipMemcpyAsync(&on, moving, 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    return KH_OK;
  };
  KH_TRY(rank());
  const bool cycles = on != 0;
  if (cycles) {  // open every cycle, then rank again
    hipLaunchKernelGGL(k_cut_cycles, dim3(grid(m)), dim3(kTB), 0, s, recs[cur].p, m, succ.p,
                       on_cycle.p);
    HIP_TRY(hipGetLastError());
    KH_TRY(rank());
    if (on) return fail(KH_EDEVICE, "contig chains did not end after opening cycles");
  }
  const Rec* A = recs[cur].p;
  // ---- placement, representatives, contig numbering and offsets
  Buf<int64_t> start_of(pool), pos_of(pool);
  Buf<uint64_t> rep_flag(pool), rep_len(pool), cidx(pool), scal(pool);
  KH_TRY(start_of.alloc(n));
  KH_TRY(pos_of.alloc(n));
  KH_TRY(rep_flag.alloc(n));
  KH_TRY(rep_len.alloc(n));
  KH_TRY(cidx.alloc(n));
  KH_TRY(scal.alloc(2));
  Buf<unsigned int> bad(pool);
  KH_TRY(bad.alloc(2));
  launch_fill_u64(reinterpret_cast<uint64_t*>(bad.p), 1, 0ull, s);
  hipLaunchKernelGGL((k_resolve<W>), dim3(grid(n)), dim3(kTB), 0, s, t->keys, n, k, A,
                     on_cycle.p, start_of.p, pos_of.p, rep_flag.p, rep_len.p, bad.p);
  HIP_TRY(hipGetLastError());
  KH_TRY(scan_exclusive(pool, rep_flag.p, cidx.p, n, scal.p, s));
  uint64_t nc = 0;
  HIP_TRY(hipMemcpyAsync(&nc, scal.p, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  Buf<uint64_t> lens(pool), offs(pool);
  KH_TRY(lens.alloc(nc + 1));
  KH_TRY(offs.alloc(nc + 1));
  hipLaunchKernelGGL(k_contig_lens, dim3(grid(n)), dim3(kTB), 0, s, rep_flag.p, cidx.p,
                     rep_len.p, n, lens.p);
  HIP_TRY(hipGetLastError());
  KH_TRY(scan_exclusive(pool, lens.p, offs.p, (int64_t)nc, scal.p + 1, s));
  uint64_t total = 0;
  HIP_TRY(hipMemcpyAsync(&total, scal.p + 1, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(offs.p + nc, scal.p + 1, 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  // ---- emission
  Buf<char> seq(pool);
  Buf<int64_t> nk(pool);
  Buf<uint64_t> depth(pool);
  Buf<uint8_t> cyc(pool);
  Buf<uint32_t> rowc(pool);
  KH_TRY(seq.alloc(total));
  KH_TRY(nk.alloc(nc));
  KH_TRY(depth.alloc(nc));
  KH_TRY(cyc.alloc(nc));
  KH_TRY(rowc.alloc(n));
  launch_fill_u64(depth.p, nc, 0ull, s);
  hipLaunchKernelGGL((k_emit<W>), dim3(grid(n)), dim3(kTB), 0, s, t->keys, t->counts, n, k, A,
                     on_cycle.p, start_of.p, pos_of.p, cidx.p, offs.p, nc, seq.p, nk.p,
                     reinterpret_cast<unsigned long long*>(depth.p), cyc.p, rowc.p, bad.p);
  HIP_TRY(hipGetLastError());
  unsigned int hbad = 0;
  HIP_TRY(hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hbad) return fail(KH_EDEVICE, "inconsistent contig chains (code %u)", hbad);
  if (cycles) {  // k-mers on cycles, for the report
    std::vector<uint8_t> h((size_t)n);
    HIP_TRY(hipMemcpy(h.data(), on_cycle.p, (size_t)n, hipMemcpyDeviceToHost));
    for (uint8_t v : h) out->cycle_kmers += v;
  }
  out->n_contigs = (int64_t)nc;
  out->total_bases = (int64_t)total;
  out->seq = seq.release();
  out->offsets = reinterpret_cast<int64_t*>(offs.release());
  out->n_kmers = nk.release();
  out->depth = depth.release();
  out->cycle = cyc.release();
  out->row_contig = rowc.release();
  out->n_rows = n;
  return KH_OK;
}

}  // namespace

int kh_scan_exclusive_u64(Pool* pool, const uint64_t* in, uint64_t* out, int64_t n,
                          uint64_t* total, hipStream_t s) {
  return scan_exclusive(pool, in, out, n, total, s);
}

static void release_contigs(kh_contigs* c) {
  if (!c->ctx) return;
  Pool& pl = c->ctx->pool;
  std::lock_guard<std::recursive_mutex> lk(pl.mu);
  pl.put(c->seq);
  pl.put(c->offsets);
  pl.put(c->n_kmers);
  pl.put(c->depth);
  pl.put(c->cycle);
  pl.put(c->row_contig);
  c->row_contig = nullptr;
  c->seq = nullptr;
  c->offsets = nullptr;
  c->n_kmers = nullptr;
  c->depth = nullptr;
  c->cycle = nullptr;
}

extern "C" int kh_traverse(kh_ctx* ctx, const kh_table* t, void* hip_stream,
                           kh_contigs** out) {
  if (!ctx || !t || !out) return fail(KH_EINVAL, "NULL argument");
  *out = nullptr;
  if (!t->ctx) return fail(KH_EINVAL, "the table's context was destroyed");
  if (t->ctx->device != ctx->device)
    return fail(KH_EINVAL, "the table lives on device %d, the context on %d", t->ctx->device,
                ctx->device);
  if (t->n_rows > (int64_t)0xfffffffe) return fail(KH_EINVAL, "too many rows");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  kh_contigs* c = new (std::nothrow) kh_contigs();
  if (!c) return fail(KH_ENOMEM, "host allocation failed");
  c->ctx = ctx;
  c->k = t->k;
  c->source = t->serial;
  int rc = KH_OK;
  if (t->n_rows == 0) {
    Buf<int64_t> off(&ctx->pool);
    rc = off.alloc(1);
    if (rc == KH_OK) {
      launch_fill_u64(reinterpret_cast<uint64_t*>(off.p), 1, 0ull, s);
      rc = hipStreamSynchronize(s) == hipSuccess ? KH_OK : fail(KH_EDEVICE, "sync failed");
      c->offsets = off.release();
    }
  } else {
    switch ((t->k + 31) / 32) {
      case 1: rc = traverse_w<1>(ctx, t, s, c); break;
      case 2: rc = traverse_w<2>(ctx, t, s, c); break;
      case 3: rc = traverse_w<3>(ctx, t, s, c); break;
      default: rc = traverse_w<4>(ctx, t, s, c); break;
    }
  }
  if (rc != KH_OK) {
    release_contigs(c);
    delete c;
    return rc;
  }
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->pool.mu);
    ctx->live_contigs.insert(c);
  }
  *out = c;
  return KH_OK;
}

extern "C" int kh_contigs_info(const kh_contigs* c, uint32_t* k, int64_t* n_contigs,
                               int64_t* total_bases, int64_t* cycle_kmers, int* rounds) {
  if (!c) return fail(KH_EINVAL, "contigs is NULL");
  if (k) *k = c->k;
  if (n_contigs) *n_contigs = c->n_contigs;
  if (total_bases) *total_bases = c->total_bases;
  if (cycle_kmers) *cycle_kmers = c->cycle_kmers;
  if (rounds) *rounds = c->rounds;
  return KH_OK;
}

extern "C" int kh_contigs_export(const kh_contigs* c, char* seq, int64_t* offsets,
                                 int64_t* n_kmers, uint64_t* depth, uint8_t* cycle,
                                 int dst_on_device) {
  if (!c) return fail(KH_EINVAL, "contigs is NULL");
  if (!c->ctx && c->n_contigs > 0) return fail(KH_EINVAL, "the contigs' context was destroyed");
  if (!c->ctx) return KH_OK;
  HIP_TRY(hipSetDevice(c->ctx->device));
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const size_t m = (size_t)c->n_contigs;
  if (seq && c->total_bases) HIP_TRY(hipMemcpy(seq, c->seq, (size_t)c->total_bases, kind));
  if (offsets) HIP_TRY(hipMemcpy(offsets, c->offsets, (m + 1) * 8, kind));
  if (m) {
    if (n_kmers) HIP_TRY(hipMemcpy(n_kmers, c->n_kmers, m * 8, kind));
    if (depth) HIP_TRY(hipMemcpy(depth, c->depth, m * 8, kind));
    if (cycle) HIP_TRY(hipMemcpy(cycle, c->cycle, m, kind));
  }
  return KH_OK;
}

extern "C" int kh_contigs_device(const kh_contigs* c, const char** seq,
                                 const int64_t** offsets) {
  if (!c) return fail(KH_EINVAL, "contigs is NULL");
  if (seq) *seq = c->seq;
  if (offsets) *offsets = c->offsets;
  return KH_OK;
}

extern "C" int kh_contigs_free(kh_contigs* c) {
  if (!c) return KH_OK;
  if (c->ctx) {
    std::lock_guard<std::recursive_mutex> lk(c->ctx->pool.mu);
    c->ctx->live_contigs.erase(c);
    release_contigs(c);
  }
  delete c;
  return KH_OK;
}

// Called by kh_destroy: the contigs' device memory goes with the context.
void kh_orphan_contigs(kh_ctx* ctx) {
  for (kh_contigs* c : ctx->live_contigs) {
    c->ctx = nullptr;
    c->n_contigs = 0;
    c->total_bases = 0;
    c->seq = nullptr;
    c->offsets = nullptr;
    c->n_kmers = nullptr;
    c->depth = nullptr;
    c->cycle = nullptr;
    c->row_contig = nullptr;
  }
  ctx->live_contigs.clear();
}
