// LSD radix sort of k-mer rows for the deterministic, key-ordered export.
//
// Reduce-then-scan per 8-bit digit: (1) each block counts the digits of its
// 3,840-row tile, (2) one exclusive scan over the digit-major table of block
// counts gives every (digit, block) its output base, (3) each block re-reads
// its tile and scatters it, ranking equal digits stably with wave ballots.
// No block ever waits on another, so the sort cannot stall.
#include "kh_internal.hpp"

namespace kh {

constexpr int kSortItems = 15;  // three blocks fit a CU's LDS (16 would fit two)
constexpr int kSortTile = kBlock * kSortItems;  // 3,840 rows per block
constexpr int kScanChunk = kBlock * 16;         // 4096 values per scan block

static inline int64_t sort_blocks(int64_t n) {
  return (n + kSortTile - 1) / kSortTile;
}

uint64_t sort_tmp_words(int64_t n) {
  const uint64_t m = 256ull * (uint64_t)sort_blocks(n);
  return m + (m + kScanChunk - 1) / kScanChunk + 64;
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_rs_hist(
    const uint64_t* __restrict__ keys, int64_t n, int word, int shift,
    uint32_t mask, uint32_t* __restrict__ hist, int64_t nblocks) {
  __shared__ uint32_t h[kBlock / 64][256];
  const int tid = threadIdx.x, wave = tid >> 6;
  for (int i = tid; i < (kBlock / 64) * 256; i += kBlock) (&h[0][0])[i] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t e = base + it * kBlock + tid;
    if (e < n) {
      const uint32_t d = (uint32_t)(keys[e * W + word] >> shift) & mask;
      atomicAdd(&h[wave][d], 1u);
    }
  }
  __syncthreads();
  {
    const int d = tid;
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += h[w][d];
    hist[(int64_t)d * nblocks + blockIdx.x] = s;
  }
}

// Exclusive scan of 16 consecutive values per thread across the block.
// Returns the block total; v is replaced by exclusive prefixes.
__device__ __forceinline__ uint32_t block_scan16(uint32_t (&v)[16],
                                                 uint32_t* lds_waves) {
  uint32_t t = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint32_t x = v[i];
    v[i] = t;
    t += x;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = t;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) lds_waves[wave] = incl;
  __syncthreads();
  uint32_t wave_off = 0, total = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    const uint32_t s = lds_waves[w];
    if (w < wave) wave_off += s;
    total += s;
  }
  const uint32_t excl = wave_off + incl - t;
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] += excl;
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(
    const uint32_t* __restrict__ x, int64_t m, uint32_t* __restrict__ part) {
  __shared__ uint32_t s[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * 16;
  uint32_t t = 0;
  for (int i = 0; i < 16; ++i)
    if (base + i < m) t += x[base + i];
  for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0;
    for (int w = 0; w < kBlock / 64; ++w) a += s[w];
    part[blockIdx.x] = a;
  }
}

// Single block: exclusive scan of the per-block partial sums.
__global__ __launch_bounds__(kBlock) void k_scan_partials(uint32_t* part,
                                                          int64_t np) {
  __shared__ uint32_t s[kBlock / 64];
  uint32_t carry = 0;
  for (int64_t c0 = 0; c0 < np; c0 += kScanChunk) {
    uint32_t v[16];
    const int64_t base = c0 + threadIdx.x * 16;
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = (base + i < np) ? part[base + i] : 0u;
    const uint32_t total = block_scan16(v, s);
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (base + i < np) part[base + i] = v[i] + carry;
    carry += total;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_down(
    uint32_t* __restrict__ x, int64_t m, const uint32_t* __restrict__ part) {
  __shared__ uint32_t s[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * 16;
  uint32_t v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = (base + i < m) ? x[base + i] : 0u;
  block_scan16(v, s);
  const uint32_t off = part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if (base + i < m) x[base + i] = v[i] + off;
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_rs_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ iin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ iout, int64_t n,
    int word, int shift, int bits, const uint32_t* __restrict__ hist,
    int64_t nblocks) {
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_wcnt[kBlock / 64][256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  s_base[tid] = hist[(int64_t)tid * nblocks + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) s_wcnt[w][tid] = 0;
  __syncthreads();
  const uint32_t mask = (1u << bits) - 1u;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t e = base + it * kBlock + tid;
    const bool valid = e < n;
    uint64_t kw[W];
    uint32_t id = 0, d = 0;
    if (valid) {
#pragma unroll
      for (int w = 0; w < W; ++w) kw[w] = kin[e * W + w];
      id = iin[e];
      d = (uint32_t)(kw[word] >> shift) & mask;
    }
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && (peers & lt) == 0) s_wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = s_base[d] + rank;
      for (int w = 0; w < wave; ++w) pos += s_wcnt[w][d];
#pragma unroll
      for (int w = 0; w < W; ++w) kout[(int64_t)pos * W + w] = kw[w];
      iout[pos] = id;
    }
    __syncthreads();
    {
      uint32_t add = 0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) {
        add += s_wcnt[w][tid];
        s_wcnt[w][tid] = 0;
      }
      s_base[tid] += add;
    }
    __syncthreads();
  }
}

// Scatter for one-word keys, staged in LDS: the tile's elements are first
// placed in LDS in digit order (stable ranks as in k_rs_scatter), then
// written out in that order, so consecutive lanes write consecutive
// addresses of a digit's run instead of 64 scattered ones.  The tile's
// count of each digit is the difference of consecutive entries of the
// scanned digit-major table (the last entry's successor is n).
__global__ __launch_bounds__(kBlock) void k_rs_scatter_lds(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ iin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ iout, int64_t n, int shift,
    int bits, const uint32_t* __restrict__ hist, int64_t nblocks) {
  __shared__ uint64_t s_key[kSortTile];
  __shared__ uint32_t s_idx[kSortTile];
  __shared__ uint32_t s_gbase[256];
  __shared__ uint32_t s_lbase[256];
  __shared__ uint32_t s_run[256];
  __shared__ uint32_t s_wcnt[kBlock / 64][256];
  __shared__ uint32_t s_scan[kBlock / 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t m = (int64_t)tid * nblocks + blockIdx.x;
  const uint32_t g = hist[m];
  const uint32_t next = m + 1 < 256 * nblocks ? hist[m + 1] : (uint32_t)n;
  s_gbase[tid] = g;
  {  // exclusive scan of the tile's digit counts (one digit per thread)
    uint32_t v[16] = {next - g};
    block_scan16(v, s_scan);  // only v[0] is non-zero: v[0] = exclusive prefix
    s_lbase[tid] = v[0];
  }
  s_run[tid] = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) s_wcnt[w][tid] = 0;
  __syncthreads();
  const uint32_t mask = (1u << bits) - 1u;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t e = base + it * kBlock + tid;
    const bool valid = e < n;
    uint64_t key = 0;
    uint32_t id = 0, d = 0;
    if (valid) {
      key = kin[e];
      id = iin[e];
      d = (uint32_t)(key >> shift) & mask;
    }
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t mb = __ballot(bit);
      peers &= bit ? mb : ~mb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && (peers & lt) == 0) s_wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = s_lbase[d] + s_run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += s_wcnt[w][d];
      s_key[pos] = key;
      s_idx[pos] = id;
    }
    __syncthreads();
    {
      uint32_t add = 0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) {
        add += s_wcnt[w][tid];
        s_wcnt[w][tid] = 0;
      }
      s_run[tid] += add;
    }
    __syncthreads();
  }
  const int64_t left = n - base;
  const int cnt = left < kSortTile ? (int)left : kSortTile;
  for (int q = tid; q < cnt; q += kBlock) {
    const uint64_t key = s_key[q];
    const uint32_t d = (uint32_t)(key >> shift) & mask;
    const uint32_t pos = s_gbase[d] + ((uint32_t)q - s_lbase[d]);
    kout[pos] = key;
    iout[pos] = s_idx[q];
  }
}

template <int W>
static void sort_pass(const uint64_t* kin, const uint32_t* iin, uint64_t* kout,
                      uint32_t* iout, int64_t n, int word, int shift, int bits,
                      uint32_t* tmp, hipStream_t s) {
  const int64_t nb = sort_blocks(n);
  const int64_t m = 256 * nb;
  uint32_t* hist = tmp;
  uint32_t* part = tmp + m;
  const int64_t np = (m + kScanChunk - 1) / kScanChunk;
  const uint32_t mask = (1u << bits) - 1u;
  hipLaunchKernelGGL(k_rs_hist<W>, dim3((unsigned)nb), dim3(kBlock), 0, s, kin,
                     n, word, shift, mask, hist, nb);
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)np), dim3(kBlock), 0, s,
                     hist, m, part);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, s, part, np);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)np), dim3(kBlock), 0, s, hist,
                     m, part);
  if (W == 1)
    hipLaunchKernelGGL(k_rs_scatter_lds, dim3((unsigned)nb), dim3(kBlock), 0, s, kin, iin,
                       kout, iout, n, shift, bits, hist, nb);
  else
    hipLaunchKernelGGL(k_rs_scatter<W>, dim3((unsigned)nb), dim3(kBlock), 0, s,
                       kin, iin, kout, iout, n, word, shift, bits, hist, nb);
}

template <int W>
static int radix_sort_w(uint64_t* ka, uint32_t* ia, uint64_t* kb, uint32_t* ib,
                        int64_t n, int bits0, uint32_t* tmp, hipStream_t s) {
  int cur = 0;
  for (int word = W - 1; word >= 0; --word) {
    const int wbits = word == 0 ? bits0 : 64;
    for (int shift = 0; shift < wbits; shift += 8) {
      const int bits = (wbits - shift) < 8 ? (wbits - shift) : 8;
      if (cur == 0) sort_pass<W>(ka, ia, kb, ib, n, word, shift, bits, tmp, s);
      else sort_pass<W>(kb, ib, ka, ia, n, word, shift, bits, tmp, s);
      cur ^= 1;
    }
  }
  return cur;
}

int radix_sort(uint64_t* ka, uint32_t* ia, uint64_t* kb, uint32_t* ib,
               int64_t n, int W, int bits0, uint32_t* tmp, hipStream_t s) {
  if (n <= 1) return 0;
  switch (W) {
    case 1: return radix_sort_w<1>(ka, ia, kb, ib, n, bits0, tmp, s);
    case 2: return radix_sort_w<2>(ka, ia, kb, ib, n, bits0, tmp, s);
    case 3: return radix_sort_w<3>(ka, ia, kb, ib, n, bits0, tmp, s);
    default: return radix_sort_w<4>(ka, ia, kb, ib, n, bits0, tmp, s);
  }
}

}  // namespace kh
