// Read localisation on the device (paper Section II, the read localisation
// subsection): after an iteration has produced contigs, reads that come from
// the same contig are brought together, so that in later iterations all
// occurrences of a k-mer arrive within a short stretch of the read stream
// and the counting table's updates hit in the caches instead of HBM.  The
// paper sends each read to the processor owning the contig it aligns to;
// here the reads are permuted in device memory.
//
// Definition (the same as the localisation oracle's): a read's anchor is the
// first of its windows, in read order, that holds k bases of A/C/G/T (either
// case) and whose canonical k-mer is a row of the walked table; the read's
// key is the contig holding that row (the traversal's row -> contig map),
// or the number of contigs when there is none.  Reads are ordered by key,
// stably.  Counting is independent of read order (Section II-A, Use case
// 1), so every table counted from the permuted reads equals the input's.
//
// Method.  One thread per read rolls the window's forward and
// reverse-complement values base by base and binary-searches the canonical
// value in the sorted rows until a window hits; an LSD radix sort over the
// key's significant bits orders the read indices.  A second call gathers
// the reads' bytes in that order (one wave per read, shared with the
// minimizer reordering).
#include <algorithm>

#include "kh_device.hpp"
#include "kh_host.hpp"
#include "kh_internal.hpp"
#include "kh_rows.hpp"

using namespace kh;

namespace {

constexpr int kLB = 256;

__device__ __forceinline__ int base_or_bad(uint8_t c) {
  switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
  }
}

template <int W>
__global__ __launch_bounds__(kLB) void k_anchor(const uint8_t* seq, const int64_t* offsets,
                                                int64_t n_reads, uint32_t k,
                                                const uint64_t* keys, int64_t n_rows,
                                                const uint32_t* row_contig, uint32_t none,
                                                uint64_t* key_out, uint32_t* idx_out) {
  const int64_t r = (int64_t)blockIdx.x * kLB + threadIdx.x;
  if (r >= n_reads) return;
  const int64_t o = offsets[r], e = offsets[r + 1];
  const int top = 2 * (int)k - 64 * (W - 1);
  uint64_t f[W], rc[W], t[W];
#pragma unroll
  for (int j = 0; j < W; ++j) f[j] = rc[j] = 0;
  uint32_t key = none, valid = 0;
  for (int64_t p = o; p < e; ++p) {
    const int b = base_or_bad(seq[p]);
    if (b < 0) {
      valid = 0;
      continue;
    }
    push_right<W>(f, b, top, t);
#pragma unroll
    for (int j = 0; j < W; ++j) f[j] = t[j];
    push_left<W>(rc, 3 - b, top, t);
#pragma unroll
    for (int j = 0; j < W; ++j) rc[j] = t[j];
    if (++valid < k) continue;
    const bool fwd = !words_less<W>(rc, f);
#pragma unroll
    for (int j = 0; j < W; ++j) t[j] = fwd ? f[j] : rc[j];
    const int64_t row = lower_bound_rows<W>(keys, n_rows, t);
    if (row < n_rows && cmp_rows<W>(keys + row * W, t) == 0) {
      key = row_contig[row];
      break;
    }
  }
  key_out[r] = key;
  idx_out[r] = (uint32_t)r;
}

// Device offsets: start at 0, never decrease (so every read lies inside
// [0, offsets[n])); bad[0] is raised otherwise.
__global__ __launch_bounds__(kLB) void k_check_offsets(const int64_t* offsets, int64_t n,
                                                       unsigned int* bad) {
  const int64_t r = (int64_t)blockIdx.x * kLB + threadIdx.x;
  if (r >= n) return;
  if ((r == 0 && offsets[0] != 0) || offsets[r + 1] < offsets[r]) atomicOr(bad, 1u);
}

// Device read offsets checked before any kernel reads a base through them.
int check_device_offsets(Pool* pool, const int64_t* offsets, int64_t n, hipStream_t s) {
  Buf<uint64_t> flag(pool);
  KH_TRY(flag.alloc(1));
  launch_fill_u64(flag.p, 1, 0ull, s);
  hipLaunchKernelGGL(k_check_offsets, dim3((unsigned)((n + kLB - 1) / kLB)), dim3(kLB), 0, s,
                     offsets, n, reinterpret_cast<unsigned int*>(flag.p));
  HIP_TRY(hipGetLastError());
  uint64_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, flag.p, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h) return fail(KH_EINVAL, "read offsets must start at 0 and never decrease");
  return KH_OK;
}

__global__ __launch_bounds__(kLB) void k_idx_to_i64(const uint32_t* idx, int64_t n,
                                                    int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * kLB + threadIdx.x;
  if (i < n) out[i] = (int64_t)idx[i];
}

unsigned lgrid(int64_t n, int per = kLB) { return (unsigned)((n + per - 1) / per); }

int bit_width(uint64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b < 1 ? 1 : b;
}

template <int W>
int localize_w(kh_ctx* ctx, const kh_table* t, const kh_contigs* c, const uint8_t* seq,
               const int64_t* offs, int64_t n, hipStream_t s, int64_t* order_dev) {
  Pool* pool = &ctx->pool;
  Buf<uint64_t> ka(pool), kb(pool);
  Buf<uint32_t> ia(pool), ib(pool), tmp(pool);
  KH_TRY(ka.alloc(n));
  KH_TRY(kb.alloc(n));
  KH_TRY(ia.alloc(n));
  KH_TRY(ib.alloc(n));
  KH_TRY(tmp.alloc(sort_tmp_words(n)));
  const uint32_t none = (uint32_t)c->n_contigs;
  hipLaunchKernelGGL((k_anchor<W>), dim3(lgrid(n)), dim3(kLB), 0, s, seq, offs, n, c->k,
                     t->keys, t->n_rows, c->row_contig, none, ka.p, ia.p);
  HIP_TRY(hipGetLastError());
  const int which = radix_sort(ka.p, ia.p, kb.p, ib.p, n, 1, bit_width(none), tmp.p, s);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_idx_to_i64, dim3(lgrid(n)), dim3(kLB), 0, s, which ? ib.p : ia.p, n,
                     order_dev);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return KH_OK;
}

}  // namespace

extern "C" int kh_localize_reads(kh_ctx* ctx, const kh_table* t, const kh_contigs* c,
                                 const kh_reads* reads, void* hip_stream, int64_t* order,
                                 int order_on_device) {
  if (!ctx || !t || !c || !reads || !order) return fail(KH_EINVAL, "NULL argument");
  if (!t->ctx || !c->ctx) return fail(KH_EINVAL, "the table's or the contigs' context was destroyed");
  if (t->ctx->device != ctx->device || c->ctx->device != ctx->device)
    return fail(KH_EINVAL, "table, contigs and context must share one device");
  if (c->source != t->serial || c->n_rows != t->n_rows || (c->n_rows > 0 && !c->row_contig))
    return fail(KH_EINVAL, "the contigs were not walked from this table");
  const int64_t n = reads->n_reads;
  if (n < 0 || (n > 0 && (!reads->seq || !reads->offsets)))
    return fail(KH_EINVAL, "bad read arrays");
  if (n > (int64_t)0xffffffff) return fail(KH_EINVAL, "too many reads");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (n == 0) return KH_OK;
  Pool* pool = &ctx->pool;
  const uint8_t* seq = reinterpret_cast<const uint8_t*>(reads->seq);
  const int64_t* offs = reads->offsets;
  Buf<uint8_t> dseq(pool);
  Buf<int64_t> doff(pool);
  if (!reads->on_device) {  // host reads: bases and offsets to the device
    if (offs[0] != 0) return fail(KH_EINVAL, "offsets[0] must be 0");
    for (int64_t r = 0; r < n; ++r)
      if (offs[r + 1] < offs[r]) return fail(KH_EINVAL, "offsets decrease at read %lld", (long long)r);
    const int64_t total = offs[n];
    KH_TRY(dseq.alloc((uint64_t)total + 1));
    KH_TRY(doff.alloc(n + 1));
    if (total) HIP_TRY(hipMemcpyAsync(dseq.p, seq, (size_t)total, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(doff.p, offs, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, s));
    seq = dseq.p;
    offs = doff.p;
  } else {
    KH_TRY(check_device_offsets(pool, offs, n, s));
  }
  Buf<int64_t> dorder(pool);
  int64_t* od = order;
  if (!order_on_device) {
    KH_TRY(dorder.alloc(n));
    od = dorder.p;
  }
  int rc;
  switch ((t->k + 31) / 32) {
    case 1: rc = localize_w<1>(ctx, t, c, seq, offs, n, s, od); break;
    case 2: rc = localize_w<2>(ctx, t, c, seq, offs, n, s, od); break;
    case 3: rc = localize_w<3>(ctx, t, c, seq, offs, n, s, od); break;
    default: rc = localize_w<4>(ctx, t, c, seq, offs, n, s, od); break;
  }
  if (rc != KH_OK) return rc;
  if (!order_on_device) HIP_TRY(hipMemcpy(order, od, (size_t)n * 8, hipMemcpyDeviceToHost));
  return KH_OK;
}

extern "C" int kh_gather_reads(kh_ctx* ctx, const kh_reads* reads, const int64_t* order,
                               void* hip_stream, char* seq_out, char* qual_out,
                               int64_t* offsets_out) {
  if (!ctx || !reads || !order || !offsets_out) return fail(KH_EINVAL, "NULL argument");
  if (!reads->on_device) return fail(KH_EINVAL, "reads must be in device memory");
  const int64_t n = reads->n_reads;
  if (n < 0 || (n > 0 && (!reads->seq || !reads->qual || !reads->offsets || !seq_out ||
                          !qual_out)))
    return fail(KH_EINVAL, "bad read arrays");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Pool* pool = &ctx->pool;
  if (n == 0) {
    launch_fill_u64(reinterpret_cast<uint64_t*>(offsets_out), 1, 0ull, s);
    HIP_TRY(hipStreamSynchronize(s));
    return KH_OK;
  }
  KH_TRY(check_device_offsets(pool, reads->offsets, n, s));
  return gather_reads_ordered(pool, reinterpret_cast<const uint8_t*>(reads->seq),
                              reinterpret_cast<const uint8_t*>(reads->qual), reads->offsets, n,
                              order, reinterpret_cast<uint8_t*>(seq_out),
                              reinterpret_cast<uint8_t*>(qual_out), offsets_out, s);
}
