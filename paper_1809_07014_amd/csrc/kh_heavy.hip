// Heavy hitters of a table (paper Section II-B: k-mers that occur so often,
// e.g. from highly abundant organisms of a metagenome, that a uniform
// distribution of the counting work would be unbalanced; the paper counts
// them with a dedicated streaming algorithm).  The counting kernels flag a
// k-mer once it reaches 4096 occurrences and recount those exactly in a
// side table, so every count is exact; this call reports the rows at or
// above a threshold explicitly: one flag pass, a prefix sum, a compaction.
#include "kh_device.hpp"
#include "kh_host.hpp"

using namespace kh;

namespace {

constexpr int kHB = 256;

__global__ __launch_bounds__(kHB) void k_heavy_flag(const uint32_t* counts, int64_t n,
                                                    uint32_t min_count, uint64_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * kHB + threadIdx.x;
  if (i < n) flag[i] = counts[i] >= min_count ? 1 : 0;
}

__global__ __launch_bounds__(kHB) void k_heavy_take(const uint64_t* keys, const uint32_t* counts,
                                                    int64_t n, int W, const uint64_t* flag,
                                                    const uint64_t* idx, uint64_t* o_keys,
                                                    uint32_t* o_counts) {
  const int64_t i = (int64_t)blockIdx.x * kHB + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const uint64_t o = idx[i];
  for (int j = 0; j < W; ++j) o_keys[o * W + j] = keys[i * W + j];
  o_counts[o] = counts[i];
}

unsigned hgrid(int64_t n) { return (unsigned)((n + kHB - 1) / kHB); }

}  // namespace

extern "C" int kh_heavy_hitters(const kh_table* t, uint32_t min_count, void* hip_stream,
                                uint64_t* keys_out, uint32_t* counts_out, int64_t cap,
                                int64_t* n_out) {
  if (!t || !n_out) return fail(KH_EINVAL, "NULL argument");
  if (cap < 0 || (cap > 0 && (!keys_out || !counts_out)))
    return fail(KH_EINVAL, "bad output buffers");
  if (min_count < 1) return fail(KH_EINVAL, "min_count must be >= 1");
  *n_out = 0;
  if (!t->ctx) {
    if (t->n_rows > 0) return fail(KH_EINVAL, "the table's context was destroyed");
    return KH_OK;
  }
  const int64_t n = t->n_rows;
  if (n == 0) return KH_OK;
  kh_ctx* ctx = t->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Pool* pool = &ctx->pool;
  const int W = (int)t->W;
  Buf<uint64_t> flag(pool), idx(pool), total(pool);
  KH_TRY(flag.alloc(n));
  KH_TRY(idx.alloc(n));
  KH_TRY(total.alloc(1));
  hipLaunchKernelGGL(k_heavy_flag, dim3(hgrid(n)), dim3(kHB), 0, s, t->counts, n, min_count,
                     flag.p);
  HIP_TRY(hipGetLastError());
  KH_TRY(kh_scan_exclusive_u64(pool, flag.p, idx.p, n, total.p, s));
  uint64_t m = 0;
  HIP_TRY(hipMemcpyAsync(&m, total.p, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *n_out = (int64_t)m;
  if (m == 0 || cap == 0) return KH_OK;
  Buf<uint64_t> ok(pool);
  Buf<uint32_t> oc(pool);
  KH_TRY(ok.alloc(m * (uint64_t)W));
  KH_TRY(oc.alloc(m));
  hipLaunchKernelGGL(k_heavy_take, dim3(hgrid(n)), dim3(kHB), 0, s, t->keys, t->counts, n, W,
                     flag.p, idx.p, ok.p, oc.p);
  HIP_TRY(hipGetLastError());
  const uint64_t take = m < (uint64_t)cap ? m : (uint64_t)cap;
  HIP_TRY(hipMemcpyAsync(keys_out, ok.p, take * W * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(counts_out, oc.p, take * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return KH_OK;
}
