// Iterative graph pruning on the device (paper Section II, the iterative
// graph pruning subsection and its Algorithm 2): a depth threshold tau
// starts at 1 and grows by the factor (1 + alpha) after every sweep while it
// stays below the largest mean depth of the remaining contigs; a sweep
// removes every contig of at most 2k bases whose mean depth is at most
// min(tau, beta * the mean depth of its neighbourhood).
//
// Definitions (the same as the pruning oracle's):
//  * depth(c) = sum of c's k-mer counts / number of its k-mers;
//  * the neighbours of c are the other contigs holding a k-mer that overlaps
//    c's first k-mer by k-1 bases on its left or c's last k-mer by k-1 bases
//    on its right (any base, either strand), each counted once;
//  * the neighbourhood's depth pools the neighbours still present: the sum
//    of their k-mers' counts / the number of their k-mers; a contig with no
//    neighbour left stays;
//  * sweeps are synchronous: a sweep decides on the contigs as they were
//    when it started and its removals take effect at its end;
//  * IEEE double, one rounding per operation: d = sum / n, nd = sum / n,
//    cut = min(tau, beta * nd), remove iff d <= cut; tau_next = tau * g with
//    g = 1 + alpha (both on the host).
//
// Method.  Only contigs of at most 2k bases can go, so only they look up
// their neighbours: the 4 + 4 overlapping k-mers of their two end k-mers are
// found in the walked table's sorted rows by binary search, and the
// traversal's row -> contig map names the contig.  The paper's parallel
// version hashes the fork k-mers into a distributed table for the same
// purpose; one GPU reads the sorted rows directly.  Each sweep is one
// grid-stride launch over all contigs (alive flags double-buffered, the
// largest remaining depth reduced per block, one atomic per block); the host
// reads back 16 bytes per sweep to run the loop.  The kept contigs are then
// compacted in their order.
#include <cmath>
#include <cstring>
#include <vector>

#include "kh_device.hpp"
#include "kh_host.hpp"
#include "kh_rows.hpp"

using namespace kh;

namespace {

constexpr int kPB = 256;
constexpr uint32_t kNone = 0xffffffffu;
constexpr unsigned kSweepBlocks = 1024;

__device__ __forceinline__ int acgt(char c) {
  switch (c) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
  }
}

// Block-wide max (bit patterns of non-negative doubles order like the
// values) and sum, one atomic of each per block.
__device__ __forceinline__ void block_flush(uint64_t mx, uint64_t cnt,
                                            unsigned long long* out) {
  __shared__ uint64_t smx[kPB / 64], scnt[kPB / 64];
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t a = __shfl_down(mx, o), b = __shfl_down(cnt, o);
    mx = a > mx ? a : mx;
    cnt += b;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    smx[wave] = mx;
    scnt[wave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kPB / 64; ++w) {
      mx = smx[w] > mx ? smx[w] : mx;
      cnt += scnt[w];
    }
    if (mx) atomicMax(&out[0], (unsigned long long)mx);
    if (cnt) atomicAdd(&out[1], (unsigned long long)cnt);
  }
}

// Contig holding k-mer t (either strand) in the walked table, or kNone.
template <int W>
__device__ __forceinline__ uint32_t holder(const uint64_t* keys, int64_t n_rows,
                                           const uint32_t* row_contig, uint32_t k,
                                           const uint64_t (&t)[W]) {
  uint64_t r[W];
  revcomp_words<W>(t, k, r);
  const bool fwd = !words_less<W>(r, t);
#pragma unroll
  for (int j = 0; j < W; ++j) r[j] = fwd ? t[j] : r[j];
  const int64_t p = lower_bound_rows<W>(keys, n_rows, r);
  if (p < n_rows && cmp_rows<W>(keys + p * W, r) == 0) return row_contig[p];
  return kNone;
}

// Per contig: mean depth, whether it is short (<= 2k bases), and for short
// contigs the distinct neighbours (up to 8, kNone-padded).  out[0] collects
// the largest mean depth; bad[0] is raised for a base outside A/C/G/T.
template <int W>
__global__ __launch_bounds__(kPB) void k_prune_setup(
    const char* seq, const int64_t* offs, const int64_t* n_kmers, const uint64_t* depth,
    int64_t nc, uint32_t k, const uint64_t* keys, int64_t n_rows, const uint32_t* row_contig,
    double* mean, uint8_t* is_short, uint32_t* nbr, unsigned long long* out,
    unsigned int* bad) {
  const int64_t c = (int64_t)blockIdx.x * kPB + threadIdx.x;
  uint64_t mx = 0;
  if (c < nc) {
    const int64_t o = offs[c], len = offs[c + 1] - o;
    const double d = (double)depth[c] / (double)n_kmers[c];
    mean[c] = d;
    mx = (uint64_t)__double_as_longlong(d);
    const bool sh = len <= 2 * (int64_t)k;
    is_short[c] = sh ? 1 : 0;
    uint32_t ids[8];
    int m = 0;
    if (sh) {
      const int top = 2 * (int)k - 64 * (W - 1);
      uint64_t f[W], l[W], t[W];
#pragma unroll
      for (int j = 0; j < W; ++j) f[j] = l[j] = 0;
      bool ok = true;
      for (uint32_t p = 0; p < k; ++p) {  // first and last k-mer, base by base
        const int a = acgt(seq[o + p]), b = acgt(seq[o + len - k + p]);
        ok = ok && a >= 0 && b >= 0;
        push_right<W>(f, a & 3, top, t);
#pragma unroll
        for (int j = 0; j < W; ++j) f[j] = t[j];
        push_right<W>(l, b & 3, top, t);
#pragma unroll
        for (int j = 0; j < W; ++j) l[j] = t[j];
      }
      if (!ok) atomicOr(bad, 1u);
      for (int b = 0; b < 4 && ok; ++b) {
        for (int side = 0; side < 2; ++side) {
          if (side == 0)
            push_left<W>(f, b, top, t);
          else
            push_right<W>(l, b, top, t);
          const uint32_t j = holder<W>(keys, n_rows, row_contig, k, t);
          if (j == kNone || j == (uint32_t)c) continue;
          if ((int64_t)j >= nc) {  // not a contig of this set: refuse
            atomicOr(bad, 2u);
            continue;
          }
          bool seen = false;
          for (int x = 0; x < m; ++x) seen = seen || ids[x] == j;
          if (!seen) ids[m++] = j;
        }
      }
    }
    for (int x = 0; x < 8; ++x) nbr[c * 8 + x] = x < m ? ids[x] : kNone;
  }
  block_flush(mx, 0, out);
}

// One sweep at threshold tau.  out[0]: largest mean depth left, out[1]:
// contigs removed.
__global__ __launch_bounds__(kPB) void k_prune_sweep(
    const double* mean, const uint8_t* is_short, const uint32_t* nbr, const uint64_t* depth,
    const int64_t* n_kmers, int64_t nc, const uint8_t* alive_in, uint8_t* alive_out,
    int32_t* removed_at, double tau, double beta, int32_t sweep, unsigned long long* out) {
#pragma clang fp contract(off)
  uint64_t mx = 0, cnt = 0;
  for (int64_t c = (int64_t)blockIdx.x * kPB + threadIdx.x; c < nc;
       c += (int64_t)gridDim.x * kPB) {
    uint8_t a = alive_in[c];
    const double d = mean[c];
    if (a && is_short[c]) {
      uint64_t sn = 0, nn = 0;
      for (int x = 0; x < 8; ++x) {
        const uint32_t j = nbr[c * 8 + x];
        if (j == kNone) break;
        if (alive_in[j]) {
          sn += depth[j];
          nn += (uint64_t)n_kmers[j];
        }
      }
      if (nn) {
        const double nd = (double)sn / (double)nn;
        const double bnd = beta * nd;
        const double cut = tau < bnd ? tau : bnd;
        if (d <= cut) {
          a = 0;
          removed_at[c] = sweep;
          ++cnt;
        }
      }
    }
    alive_out[c] = a;
    if (a) {
      const uint64_t bits = (uint64_t)__double_as_longlong(d);
      mx = bits > mx ? bits : mx;
    }
  }
  block_flush(mx, cnt, out);
}

__global__ __launch_bounds__(kPB) void k_prune_keep(const uint8_t* alive, const int64_t* offs,
                                                    int64_t nc, uint64_t* keep,
                                                    uint64_t* lens) {
  const int64_t c = (int64_t)blockIdx.x * kPB + threadIdx.x;
  if (c >= nc) return;
  keep[c] = alive[c] ? 1 : 0;
  lens[c] = alive[c] ? (uint64_t)(offs[c + 1] - offs[c]) : 0;
}

// Kept contigs to their new index; out[0] collects the k-mers on cycles.
__global__ __launch_bounds__(kPB) void k_prune_place(
    const uint8_t* alive, const int64_t* n_kmers, const uint64_t* depth, const uint8_t* cycle,
    int64_t nc, const uint64_t* idx, const uint64_t* noff, int64_t* o_off, int64_t* o_nk,
    uint64_t* o_depth, uint8_t* o_cycle, unsigned long long* out) {
  const int64_t c = (int64_t)blockIdx.x * kPB + threadIdx.x;
  if (c >= nc || !alive[c]) return;
  const uint64_t i = idx[c];
  o_off[i] = (int64_t)noff[c];
  o_nk[i] = n_kmers[c];
  o_depth[i] = depth[c];
  o_cycle[i] = cycle[c];
  if (cycle[c]) atomicAdd(&out[0], (unsigned long long)n_kmers[c]);
}

// One wave per contig copies its bases.
__global__ __launch_bounds__(kPB) void k_prune_copy(const uint8_t* alive, const int64_t* offs,
                                                    int64_t nc, const uint64_t* noff,
                                                    const char* seq, char* o_seq) {
  const int64_t c = (int64_t)blockIdx.x * (kPB / 64) + (threadIdx.x >> 6);
  if (c >= nc || !alive[c]) return;
  const int64_t o = offs[c], len = offs[c + 1] - o, n = (int64_t)noff[c];
  for (int64_t p = threadIdx.x & 63; p < len; p += 64) o_seq[n + p] = seq[o + p];
}

unsigned pgrid(int64_t n, int per_block = kPB) {
  return (unsigned)((n + per_block - 1) / per_block);
}

double from_bits(uint64_t b) {
  double d;
  std::memcpy(&d, &b, 8);
  return d;
}

template <int W>
int prune_w(kh_ctx* ctx, const kh_table* t, const kh_contigs* c, double alpha, double beta,
            hipStream_t s, kh_contigs* res, int32_t* removed_host, kh_prune_report* rep) {
  Pool* pool = &ctx->pool;
  const int64_t nc = c->n_contigs;
  const uint32_t k = c->k;
  Buf<double> mean(pool);
  Buf<uint8_t> is_short(pool), alive[2] = {Buf<uint8_t>(pool), Buf<uint8_t>(pool)};
  Buf<uint32_t> nbr(pool);
  Buf<int32_t> removed(pool);
  Buf<uint64_t> scal(pool);
  KH_TRY(mean.alloc(nc));
  KH_TRY(is_short.alloc(nc));
  KH_TRY(alive[0].alloc(nc + 8));
  KH_TRY(alive[1].alloc(nc + 8));
  KH_TRY(nbr.alloc((uint64_t)nc * 8));
  KH_TRY(removed.alloc(nc + 2));
  KH_TRY(scal.alloc(4));
  unsigned long long* out = reinterpret_cast<unsigned long long*>(scal.p);
  unsigned int* bad = reinterpret_cast<unsigned int*>(scal.p + 3);
  launch_fill_u64(scal.p, 4, 0ull, s);
  launch_fill_u64(reinterpret_cast<uint64_t*>(removed.p), (nc + 2) / 2, ~0ull, s);
  launch_fill_u64(reinterpret_cast<uint64_t*>(alive[0].p), (nc + 8) / 8, 0x0101010101010101ull,
                  s);
  hipLaunchKernelGGL((k_prune_setup<W>), dim3(pgrid(nc)), dim3(kPB), 0, s, c->seq, c->offsets,
                     c->n_kmers, c->depth, nc, k, t->keys, t->n_rows, c->row_contig, mean.p,
                     is_short.p, nbr.p, out, bad);
  HIP_TRY(hipGetLastError());
  uint64_t h[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(h, scal.p, 32, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h[3] & 1) return fail(KH_EINVAL, "a contig holds a base other than A/C/G/T");
  if (h[3]) return fail(KH_EDEVICE, "row -> contig map out of range");
  // ---- Algorithm 2's loop
  const double g = 1.0 + alpha;
  double tau = 1.0, md = from_bits(h[0]);
  int64_t sweeps = 0, n_removed = 0;
  int cur = 0;
  while (tau < md) {
    if (sweeps >= 0x7fffffff) return fail(KH_EINVAL, "too many sweeps");
    launch_fill_u64(scal.p, 2, 0ull, s);
    hipLaunchKernelGGL(k_prune_sweep, dim3(std::min<unsigned>(kSweepBlocks, pgrid(nc))),
                       dim3(kPB), 0, s, mean.p, is_short.p, nbr.p, c->depth, c->n_kmers, nc,
                       alive[cur].p, alive[cur ^ 1].p, removed.p, tau, beta, (int32_t)sweeps,
                       out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h, scal.p, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    md = from_bits(h[0]);
    n_removed += (int64_t)h[1];
    cur ^= 1;
    ++sweeps;
    tau = tau * g;
  }
  if (removed_host)
    HIP_TRY(hipMemcpy(removed_host, removed.p, (size_t)nc * 4, hipMemcpyDeviceToHost));
  // ---- compaction of the kept contigs, in their order
  const uint8_t* al = alive[cur].p;
  Buf<uint64_t> keep(pool), lens(pool), idx(pool), noff(pool);
  KH_TRY(keep.alloc(nc));
  KH_TRY(lens.alloc(nc));
  KH_TRY(idx.alloc(nc));
  KH_TRY(noff.alloc(nc));
  hipLaunchKernelGGL(k_prune_keep, dim3(pgrid(nc)), dim3(kPB), 0, s, al, c->offsets, nc, keep.p,
                     lens.p);
  HIP_TRY(hipGetLastError());
  KH_TRY(kh_scan_exclusive_u64(pool, keep.p, idx.p, nc, scal.p, s));
  KH_TRY(kh_scan_exclusive_u64(pool, lens.p, noff.p, nc, scal.p + 1, s));
  HIP_TRY(hipMemcpyAsync(h, scal.p, 16, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t kept = (int64_t)h[0], bases = (int64_t)h[1];
  Buf<char> o_seq(pool);
  Buf<int64_t> o_off(pool), o_nk(pool);
  Buf<uint64_t> o_depth(pool);
  Buf<uint8_t> o_cycle(pool);
  KH_TRY(o_seq.alloc(bases));
  KH_TRY(o_off.alloc(kept + 1));
  KH_TRY(o_nk.alloc(kept));
  KH_TRY(o_depth.alloc(kept));
  KH_TRY(o_cycle.alloc(kept));
  HIP_TRY(hipMemcpyAsync(o_off.p + kept, scal.p + 1, 8, hipMemcpyDeviceToDevice, s));
  launch_fill_u64(scal.p + 2, 1, 0ull, s);
  hipLaunchKernelGGL(k_prune_place, dim3(pgrid(nc)), dim3(kPB), 0, s, al, c->n_kmers, c->depth,
                     c->cycle, nc, idx.p, noff.p, o_off.p, o_nk.p, o_depth.p, o_cycle.p,
                     out + 2);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_prune_copy, dim3(pgrid(nc, kPB / 64)), dim3(kPB), 0, s, al, c->offsets,
                     nc, noff.p, c->seq, o_seq.p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h + 2, scal.p + 2, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  res->n_contigs = kept;
  res->total_bases = bases;
  res->cycle_kmers = (int64_t)h[2];
  res->seq = o_seq.release();
  res->offsets = o_off.release();
  res->n_kmers = o_nk.release();
  res->depth = o_depth.release();
  res->cycle = o_cycle.release();
  if (rep) {
    rep->sweeps = sweeps;
    rep->removed = n_removed;
    rep->tau = tau;
    rep->max_depth = md;
  }
  return KH_OK;
}

}  // namespace

extern "C" void kh_default_prune_params(kh_prune_params* p) {
  if (!p) return;
  p->alpha = 0.1;
  p->beta = 0.2;
}

extern "C" int kh_prune(kh_ctx* ctx, const kh_table* t, const kh_contigs* c,
                        const kh_prune_params* params, void* hip_stream, kh_contigs** out,
                        int32_t* removed_at, kh_prune_report* report) {
  if (!ctx || !t || !c || !out) return fail(KH_EINVAL, "NULL argument");
  *out = nullptr;
  kh_prune_params p;
  kh_default_prune_params(&p);
  if (params) p = *params;
  if (!(p.alpha >= 1e-3 && p.alpha <= 1e3))
    return fail(KH_EINVAL, "alpha must lie in [0.001, 1000]");
  if (!(p.beta >= 0.0 && p.beta <= 1e6)) return fail(KH_EINVAL, "beta must lie in [0, 1e6]");
  if (!t->ctx || !c->ctx) return fail(KH_EINVAL, "the table's or the contigs' context was destroyed");
  if (t->ctx->device != ctx->device || c->ctx->device != ctx->device)
    return fail(KH_EINVAL, "table, contigs and context must share one device");
  if (c->source != t->serial || c->n_rows != t->n_rows || (c->n_rows > 0 && !c->row_contig))
    return fail(KH_EINVAL, "the contigs were not walked from this table");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  kh_contigs* r = new (std::nothrow) kh_contigs();
  if (!r) return fail(KH_ENOMEM, "host allocation failed");
  r->ctx = ctx;
  r->k = c->k;
  int rc = KH_OK;
  if (c->n_contigs == 0) {
    Buf<int64_t> off(&ctx->pool);
    rc = off.alloc(1);
    if (rc == KH_OK) {
      launch_fill_u64(reinterpret_cast<uint64_t*>(off.p), 1, 0ull, s);
      rc = hipStreamSynchronize(s) == hipSuccess ? KH_OK : fail(KH_EDEVICE, "sync failed");
      r->offsets = off.release();
    }
    if (report) *report = kh_prune_report{0, 0, 1.0, 0.0};
  } else {
    switch ((c->k + 31) / 32) {
      case 1: rc = prune_w<1>(ctx, t, c, p.alpha, p.beta, s, r, removed_at, report); break;
      case 2: rc = prune_w<2>(ctx, t, c, p.alpha, p.beta, s, r, removed_at, report); break;
      case 3: rc = prune_w<3>(ctx, t, c, p.alpha, p.beta, s, r, removed_at, report); break;
      default: rc = prune_w<4>(ctx, t, c, p.alpha, p.beta, s, r, removed_at, report); break;
    }
  }
  if (rc != KH_OK) {
    kh_contigs_free(r);
    return rc;
  }
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->pool.mu);
    ctx->live_contigs.insert(r);
  }
  *out = r;
  return KH_OK;
}
