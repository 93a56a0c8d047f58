// Merging the k-mers of earlier contigs into a k-mer table (paper Section
// II, Algorithm 1's Merge step, and the subsection on merging k-mer sets):
// contigs assembled with a smaller k contribute every one of their k-mers as
// an error-free k-mer with unique high-quality extensions; a k-mer already
// in the table keeps its row (the reads' k-mers are stored first), a new
// one becomes a row with count 0 whose code per side is the neighbouring
// contig base when all its occurrences have one and agree, 'X' when none
// has one, 'F' otherwise.
//
// Method.  The contigs are counted as reads whose every base is of high
// quality (kh_count with min_count 1): that gives each contig k-mer its
// number of occurrences and its neighbouring-base tallies, from which the
// rule above follows (an occurrence lacks a left neighbour iff the count
// exceeds the left tallies' sum).  The two sorted row sets are then merged:
// every row finds its place by a binary search in the other set, contig
// rows whose key is a table row are dropped, and a prefix sum numbers the
// kept ones.
#include <algorithm>
#include <vector>

#include "kh_device.hpp"
#include "kh_host.hpp"
#include "kh_rows.hpp"

using namespace kh;

namespace {

constexpr int kMB = 256;

// Contig rows: place in the table, and whether the key is new.
template <int W>
__global__ __launch_bounds__(kMB) void k_merge_probe(const uint64_t* tkeys, int64_t nt,
                                                     const uint64_t* ckeys, int64_t nc,
                                                     int64_t* cpos, uint64_t* keep) {
  const int64_t j = (int64_t)blockIdx.x * kMB + threadIdx.x;
  if (j >= nc) return;
  const uint64_t* q = ckeys + j * W;
  const int64_t p = lower_bound_rows<W>(tkeys, nt, q);
  cpos[j] = p;
  keep[j] = (p < nt && cmp_rows<W>(tkeys + p * W, q) == 0) ? 0 : 1;
}

__device__ __forceinline__ uint8_t contig_side(const uint32_t* tallies, uint32_t count) {
  uint32_t sum = 0, nb = 0, which = 0;
  for (int b = 0; b < 4; ++b) {
    sum += tallies[b];
    if (tallies[b]) {
      ++nb;
      which = (uint32_t)b;
    }
  }
  if (nb == 0) return 'X';
  if (nb == 1 && sum == count) return (uint8_t)"ACGT"[which];
  return 'F';
}

// Table rows keep their record; each moves up by the new contig rows before it.
template <int W>
__global__ __launch_bounds__(kMB) void k_merge_place_table(
    const uint64_t* tkeys, const uint32_t* tcounts, const uint32_t* text, const uint8_t* tcodes,
    int64_t nt, const uint64_t* ckeys, int64_t nc, const uint64_t* kept_before,
    uint64_t* okeys, uint32_t* ocounts, uint32_t* oext, uint8_t* ocodes) {
  const int64_t i = (int64_t)blockIdx.x * kMB + threadIdx.x;
  if (i >= nt) return;
  const int64_t lb = lower_bound_rows<W>(ckeys, nc, tkeys + i * W);
  const int64_t o = i + (int64_t)kept_before[lb];
#pragma unroll
  for (int j = 0; j < W; ++j) okeys[o * W + j] = tkeys[i * W + j];
  ocounts[o] = tcounts[i];
#pragma unroll
  for (int j = 0; j < 8; ++j) oext[o * 8 + j] = text[i * 8 + j];
  ocodes[2 * o] = tcodes[2 * i];
  ocodes[2 * o + 1] = tcodes[2 * i + 1];
}

// New contig rows: count 0, no tallies, codes from the contig neighbours.
template <int W>
__global__ __launch_bounds__(kMB) void k_merge_place_contigs(
    const uint64_t* ckeys, const uint32_t* ccounts, const uint32_t* cext, int64_t nc,
    const int64_t* cpos, const uint64_t* keep, const uint64_t* kept_before, uint64_t* okeys,
    uint32_t* ocounts, uint32_t* oext, uint8_t* ocodes) {
  const int64_t j = (int64_t)blockIdx.x * kMB + threadIdx.x;
  if (j >= nc || !keep[j]) return;
  const int64_t o = cpos[j] + (int64_t)kept_before[j];
#pragma unroll
  for (int w = 0; w < W; ++w) okeys[o * W + w] = ckeys[j * W + w];
  ocounts[o] = 0;
#pragma unroll
  for (int x = 0; x < 8; ++x) oext[o * 8 + x] = 0;
  ocodes[2 * o] = contig_side(cext + j * 8, ccounts[j]);
  ocodes[2 * o + 1] = contig_side(cext + j * 8 + 4, ccounts[j]);
}

__global__ void k_zero_bytes(uint8_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kMB + threadIdx.x;
  if (i < n) p[i] = 0;
}

unsigned mgrid(int64_t n) { return (unsigned)((n + kMB - 1) / kMB); }

template <int W>
int merge_rows(kh_ctx* ctx, const kh_table* t, const kh_table* c, hipStream_t s,
               kh_table* out) {
  Pool* pool = &ctx->pool;
  const int64_t nt = t->n_rows, nc = c->n_rows;
  Buf<int64_t> cpos(pool);
  Buf<uint64_t> keep(pool), before(pool), total(pool);
  KH_TRY(cpos.alloc(nc + 1));
  KH_TRY(keep.alloc(nc + 1));
  KH_TRY(before.alloc(nc + 1));
  KH_TRY(total.alloc(1));
  if (nc > 0) {
    hipLaunchKernelGGL((k_merge_probe<W>), dim3(mgrid(nc)), dim3(kMB), 0, s, t->keys, nt,
                       c->keys, nc, cpos.p, keep.p);
    HIP_TRY(hipGetLastError());
  }
  KH_TRY(kh_scan_exclusive_u64(pool, keep.p, before.p, nc, total.p, s));
  // before[nc] = kept rows in all (table rows past the last contig row)
  HIP_TRY(hipMemcpyAsync(before.p + nc, total.p, 8, hipMemcpyDeviceToDevice, s));
  uint64_t added = 0;
  HIP_TRY(hipMemcpyAsync(&added, total.p, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t n = nt + (int64_t)added;
  Buf<uint64_t> keys(pool);
  Buf<uint32_t> counts(pool), ext(pool);
  Buf<uint8_t> codes(pool);
  KH_TRY(keys.alloc((uint64_t)n * W));
  KH_TRY(counts.alloc((uint64_t)n));
  KH_TRY(ext.alloc((uint64_t)n * 8));
  KH_TRY(codes.alloc((uint64_t)n * 2));
  if (nt > 0) {
    hipLaunchKernelGGL((k_merge_place_table<W>), dim3(mgrid(nt)), dim3(kMB), 0, s, t->keys,
                       t->counts, t->ext, t->codes, nt, c->keys, nc, before.p, keys.p,
                       counts.p, ext.p, codes.p);
    HIP_TRY(hipGetLastError());
  }
  if (nc > 0) {
    hipLaunchKernelGGL((k_merge_place_contigs<W>), dim3(mgrid(nc)), dim3(kMB), 0, s, c->keys,
                       c->counts, c->ext, nc, cpos.p, keep.p, before.p, keys.p, counts.p,
                       ext.p, codes.p);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(s));
  out->n_rows = n;
  out->n_windows = t->n_windows;
  out->keys = keys.release();
  out->counts = counts.release();
  out->ext = ext.release();
  out->codes = codes.release();
  return KH_OK;
}

}  // namespace

extern "C" int kh_merge_contigs(kh_ctx* ctx, const kh_table* t, const char* seq,
                                const int64_t* offsets, int64_t n_contigs, int on_device,
                                void* hip_stream, kh_table** out) {
  if (!ctx || !t || !out) return fail(KH_EINVAL, "NULL argument");
  *out = nullptr;
  if (!t->ctx) return fail(KH_EINVAL, "the table's context was destroyed");
  if (t->ctx->device != ctx->device)
    return fail(KH_EINVAL, "the table lives on device %d, the context on %d", t->ctx->device,
                ctx->device);
  if (n_contigs < 0 || (n_contigs > 0 && (!seq || !offsets)))
    return fail(KH_EINVAL, "bad contig arrays");
  if (t->k % 2 == 0) return fail(KH_EINVAL, "k must be odd");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // ---- the contigs' k-mers, counted as reads of high quality everywhere
  int64_t total = 0;
  if (n_contigs > 0) {
    if (on_device) {
      HIP_TRY(hipMemcpyAsync(&total, offsets + n_contigs, 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
    } else {
      total = offsets[n_contigs];
    }
  }
  std::vector<uint8_t> hq;
  Buf<uint8_t> dq(&ctx->pool);
  kh_reads r{};
  r.seq = seq;
  r.offsets = offsets;
  r.n_reads = n_contigs;
  r.on_device = on_device ? 1 : 0;
  if (on_device) {
    KH_TRY(dq.alloc((uint64_t)total + 1));
    hipLaunchKernelGGL(k_zero_bytes, dim3(mgrid(total + 1)), dim3(kMB), 0, s, dq.p, total + 1);
    HIP_TRY(hipGetLastError());
    r.qual = reinterpret_cast<const char*>(dq.p);
  } else {
    hq.assign((size_t)total + 1, 0);
    r.qual = reinterpret_cast<const char*>(hq.data());
  }
  kh_params p;
  kh_default_params(&p, t->k);
  p.min_count = 1;
  p.qual_offset = 0;  // every quality byte is 0 and the cutoff 0: all bases count
  p.qual_cutoff = 0;
  p.load_factor = 0.7f;  // contig k-mers are nearly all distinct: plan for their count
  // Contig k-mers are nearly all distinct (a row per window), which the
  // single-table path counts with one update per window; the owner path
  // would gain nothing from its LDS tables and stage a row per window.
  kh_table* c = nullptr;
  {
    const uint32_t partitioned = ctx->tune.partitioned;
    ctx->tune.partitioned = 0;
    const int crc = kh_count(ctx, &r, &p, hip_stream, &c);
    ctx->tune.partitioned = partitioned;
    KH_TRY(crc);
  }
  kh_table* m = nullptr;
  int rc = make_table(ctx, t->k, &m);
  if (rc == KH_OK) {
    switch ((t->k + 31) / 32) {
      case 1: rc = merge_rows<1>(ctx, t, c, s, m); break;
      case 2: rc = merge_rows<2>(ctx, t, c, s, m); break;
      case 3: rc = merge_rows<3>(ctx, t, c, s, m); break;
      default: rc = merge_rows<4>(ctx, t, c, s, m); break;
    }
  }
  kh_table_free(c);
  if (rc != KH_OK) {
    kh_table_free(m);
    return rc;
  }
  *out = m;
  return KH_OK;
}
