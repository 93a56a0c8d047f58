// Read reordering shared by read localisation and the aggregating counting
// pass: gathering reads in a given order, and an order that needs no
// contigs -- reads sorted by their minimizer (the smallest hash of their
// canonical 15-mers), which brings reads that overlap on the genome, and so
// share k-mers, next to each other.  Counting does not depend on read order
// (Section II-A, Use case 1), so neither changes a table.
#include "kh_device.hpp"
#include "kh_host.hpp"
#include "kh_internal.hpp"

namespace kh {

namespace {

constexpr int kRB = 256;
constexpr int kMinimizerLen = 15;  // 30 bits of 2-bit codes

__device__ __forceinline__ int base_code(uint8_t c) {
  switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
  }
}

// One thread per read: the top 32 bits of the smallest mixed canonical
// 15-mer (all ones for a read without one), and the read's index.  The
// block's reads are contiguous, so their bytes are first copied into LDS
// with coalesced loads when they fit (else read from global memory).
// Offsets that decrease, start elsewhere than 0 or pass n raise bad[0];
// such a read's bases are not read.
constexpr int kStageBytes = 40960;

__global__ __launch_bounds__(kRB) void k_read_minimizer(const uint8_t* seq, const int64_t* off,
                                                        int64_t n_reads, int64_t n,
                                                        uint64_t* key, uint32_t* idx,
                                                        unsigned int* bad) {
  __shared__ uint8_t s_seq[kStageBytes];
  __shared__ int s_ok;
  const int64_t r0 = (int64_t)blockIdx.x * kRB;
  const int64_t r_last = min(n_reads, r0 + kRB);  // one past the block's last read
  const int64_t r = r0 + threadIdx.x;
  // the block's byte range, if its offsets are sane
  const int64_t lo = off[r0], hi = off[r_last];
  if (threadIdx.x == 0) s_ok = lo >= 0 && hi >= lo && hi <= n && hi - lo <= kStageBytes;
  __syncthreads();
  const bool staged = s_ok != 0;
  if (staged)
    for (int64_t i = threadIdx.x; i < hi - lo; i += kRB) s_seq[i] = seq[lo + i];
  __syncthreads();
  if (r >= n_reads) return;
  idx[r] = (uint32_t)r;
  const int64_t a = off[r], b = off[r + 1];
  if (a < 0 || b < a || b > n || (r == 0 && a != 0)) {
    atomicOr(bad, 1u);
    key[r] = 0xffffffffull;
    return;
  }
  constexpr uint32_t kMask = (1u << (2 * kMinimizerLen)) - 1u;
  uint32_t f = 0, rc = 0;
  int valid = 0;
  uint64_t best = ~0ull;
  const bool in_lds = staged && a >= lo && b <= hi;
  for (int64_t p = a; p < b; ++p) {
    const int c = base_code(in_lds ? s_seq[p - lo] : seq[p]);
    if (c < 0) {
      valid = 0;
      continue;
    }
    f = ((f << 2) | (uint32_t)c) & kMask;
    rc = (rc >> 2) | ((uint32_t)(3 - c) << (2 * kMinimizerLen - 2));
    if (++valid >= kMinimizerLen) {
      const uint64_t h = fmix64((uint64_t)(f < rc ? f : rc) ^ 0x9e3779b97f4a7c15ull);
      best = h < best ? h : best;
    }
  }
  key[r] = best >> 32;
}

__global__ __launch_bounds__(kRB) void k_idx_to_i64(const uint32_t* idx, int64_t n,
                                                    int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * kRB + threadIdx.x;
  if (i < n) out[i] = (int64_t)idx[i];
}

// Lengths of the reads in their new order; bad[0] is raised for an index
// out of range.
__global__ __launch_bounds__(kRB) void k_order_lens(const int64_t* offsets, int64_t n,
                                                    const int64_t* order, uint64_t* lens,
                                                    unsigned int* bad) {
  const int64_t i = (int64_t)blockIdx.x * kRB + threadIdx.x;
  if (i >= n) return;
  const int64_t r = order[i];
  if (r < 0 || r >= n) {
    atomicOr(bad, 1u);
    lens[i] = 0;
    return;
  }
  lens[i] = (uint64_t)(offsets[r + 1] - offsets[r]);
}

// One wave per read copies its bases and qualities to its new place.
__global__ __launch_bounds__(kRB) void k_gather_bytes(const uint8_t* seq, const uint8_t* qual,
                                                      const int64_t* offsets, int64_t n,
                                                      const int64_t* order,
                                                      const int64_t* new_off, uint8_t* o_seq,
                                                      uint8_t* o_qual) {
  const int64_t i = (int64_t)blockIdx.x * (kRB / 64) + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t r = order[i];
  const int64_t src = offsets[r], len = offsets[r + 1] - src, dst = new_off[i];
  for (int64_t p = threadIdx.x & 63; p < len; p += 64) {
    o_seq[dst + p] = seq[src + p];
    o_qual[dst + p] = qual[src + p];
  }
}

unsigned rgrid(int64_t n, int per = kRB) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int gather_reads_ordered(Pool* pool, const uint8_t* seq, const uint8_t* qual,
                         const int64_t* offsets, int64_t n_reads, const int64_t* order,
                         uint8_t* o_seq, uint8_t* o_qual, int64_t* o_off, hipStream_t s) {
  if (n_reads == 0) {
    launch_fill_u64(reinterpret_cast<uint64_t*>(o_off), 1, 0ull, s);
    HIP_TRY(hipStreamSynchronize(s));
    return KH_OK;
  }
  Buf<uint64_t> lens(pool), scal(pool);
  KH_TRY(lens.alloc(n_reads));
  KH_TRY(scal.alloc(2));
  launch_fill_u64(scal.p, 2, 0ull, s);
  hipLaunchKernelGGL(k_order_lens, dim3(rgrid(n_reads)), dim3(kRB), 0, s, offsets, n_reads,
                     order, lens.p, reinterpret_cast<unsigned int*>(scal.p + 1));
  HIP_TRY(hipGetLastError());
  KH_TRY(kh_scan_exclusive_u64(pool, lens.p, reinterpret_cast<uint64_t*>(o_off), n_reads,
                               scal.p, s));
  uint64_t h[2] = {0, 0};
  int64_t total = 0;
  HIP_TRY(hipMemcpyAsync(h, scal.p, 16, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&total, offsets + n_reads, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h[1]) return fail(KH_EINVAL, "order holds a read index out of range");
  if ((int64_t)h[0] != total)
    return fail(KH_EINVAL, "order is not a permutation (bases %llu, expected %lld)",
                (unsigned long long)h[0], (long long)total);
  HIP_TRY(hipMemcpyAsync(o_off + n_reads, scal.p, 8, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_gather_bytes, dim3(rgrid(n_reads, kRB / 64)), dim3(kRB), 0, s, seq, qual,
                     offsets, n_reads, order, o_off, o_seq, o_qual);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return KH_OK;
}

int reorder_by_minimizer(Pool* pool, const uint8_t* seq, const uint8_t* qual,
                         const int64_t* offsets, int64_t n_reads, int64_t n, hipStream_t s,
                         uint8_t* o_seq, uint8_t* o_qual, int64_t* o_off) {
  if (n_reads > (int64_t)0xffffffff) return fail(KH_EINVAL, "too many reads");
  Buf<uint64_t> ka(pool), kb(pool), flag(pool);
  Buf<uint32_t> ia(pool), ib(pool), tmp(pool);
  Buf<int64_t> order(pool);
  KH_TRY(ka.alloc(n_reads));
  KH_TRY(kb.alloc(n_reads));
  KH_TRY(ia.alloc(n_reads));
  KH_TRY(ib.alloc(n_reads));
  KH_TRY(tmp.alloc(sort_tmp_words(n_reads)));
  KH_TRY(order.alloc(n_reads));
  KH_TRY(flag.alloc(1));
  launch_fill_u64(flag.p, 1, 0ull, s);
  hipLaunchKernelGGL(k_read_minimizer, dim3(rgrid(n_reads)), dim3(kRB), 0, s, seq, offsets,
                     n_reads, n, ka.p, ia.p, reinterpret_cast<unsigned int*>(flag.p));
  HIP_TRY(hipGetLastError());
  uint64_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, flag.p, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (bad) return fail(KH_EINVAL, "offsets are not non-decreasing from 0 to the base count");
  const int which = radix_sort(ka.p, ia.p, kb.p, ib.p, n_reads, 1, 32, tmp.p, s);
  hipLaunchKernelGGL(k_idx_to_i64, dim3(rgrid(n_reads)), dim3(kRB), 0, s,
                     which ? ib.p : ia.p, n_reads, order.p);
  HIP_TRY(hipGetLastError());
  return gather_reads_ordered(pool, seq, qual, offsets, n_reads, order.p, o_seq, o_qual, o_off,
                              s);
}

}  // namespace kh
