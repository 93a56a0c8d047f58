// LSD radix sort of k-mer rows for the deterministic, key-ordered export.
//
// Reduce-then-scan per 8-bit digit: (1) each block counts the digits of its
// 3,840-row tile, (2) one exclusive scan over the digit-major table of block
// counts gives every (digit, block) its output base, (3) each block re-reads
// its tile and scatters it, ranking equal digits stably with wave ballots.
// No block ever waits on another, so the sort cannot stall.
#include <vector>

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

uint64_t scan_tmp_words(int64_t m) {
  return (uint64_t)((m + kScanChunk - 1) / kScanChunk) + 64;
}

void exclusive_scan_u32(uint32_t* x, int64_t m, uint32_t* part, hipStream_t s) {
  if (m <= 0) return;
  const int64_t np = (m + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)np), dim3(kBlock), 0, s, x, m, part);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, s, part, np);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)np), dim3(kBlock), 0, s, x, m, part);
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

// ------------------------------------------------- segmented row sort ----
//
// Rows sorted by one key word of `bits` bits in three steps: two stable LSD
// passes over the top B bits (B <= 16) put the rows in the order of those
// bits, a pass over the rows marks where each of the 2^B buckets starts, and
// runs of consecutive buckets holding at most kSegCap rows (segments) are
// each sorted by the remaining bits in LDS by one workgroup.  A row then
// crosses device memory about three times instead of once per 8-bit digit.
// A set of at most kSegCap rows is one segment, sorted by one launch.
// A bucket larger than a segment (rare: bucket sizes stay within a few times
// their mean for k-mer keys) is sorted by the plain LSD passes on its range.

constexpr int kSegThreads = 1024;
constexpr int kSegWaves = kSegThreads / 64;
constexpr int kSegCap = 16384;    // rows of a segment (its u64 values: 128 KiB of LDS)
constexpr int kSegPosBits = 14;   // a row's place in its segment
constexpr int kSegItems = kSegCap / kSegThreads;
constexpr int kSegMaxKeyBits = 64 - kSegPosBits;
constexpr int kSegDigit = 5;      // key bits per LDS pass
constexpr int kSegBins = 1 << kSegDigit;
constexpr int kSegCounters = kSegBins * kSegItems * kSegWaves;  // 8,192

struct SortSeg {
  int64_t r0;     // first row
  int32_t n;      // rows
  int32_t nb;     // significant bits of key - base over the segment
  uint64_t base;  // key of the segment's first bucket's first value
};

// Each value in LDS is ((key - base) << kSegPosBits) | (row - r0): sorting
// the values orders the rows by key, and the low bits name the row whose
// payload follows it.  LSD passes of 5-bit digits.  In a pass, value i
// (i = it * 1,024 + wave * 64 + lane) is ranked among the values of its
// wave and iteration with the same digit by wave ballots, the leader of
// each digit group writes the group's size to a counter indexed (digit,
// iteration, wave), one block-wide exclusive scan over the counters in that
// order gives every group its first position, and each value goes to its
// group's position plus its rank: a stable pass with four barriers.  The
// values of a pass are held in registers, so one LDS buffer serves as both
// source and destination.  `segs` null: the one segment `one`.
__global__ __launch_bounds__(kSegThreads) void k_seg_sort(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ iin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ iout,
    const SortSeg* __restrict__ segs, SortSeg one) {
  __shared__ uint64_t v[kSegCap];
  __shared__ uint16_t cnt[kSegCounters];
  __shared__ uint32_t s_part[kSegWaves];
  const SortSeg sg = segs ? segs[blockIdx.x] : one;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int n = sg.n;
  for (int i = tid; i < n; i += kSegThreads)
    v[i] = ((kin[sg.r0 + i] - sg.base) << kSegPosBits) | (uint64_t)i;
  const int end = kSegPosBits + sg.nb;
  for (int shift = kSegPosBits; shift < end; shift += kSegDigit) {
    const int bits = end - shift < kSegDigit ? end - shift : kSegDigit;
    const uint32_t mask = (1u << bits) - 1u;
    __syncthreads();  // v holds the previous pass's order
    uint64_t x[kSegItems];
    uint32_t rk[kSegItems];
#pragma unroll
    for (int it = 0; it < kSegItems; ++it) {
      const int e = it * kSegThreads + tid;
      x[it] = e < n ? v[e] : 0ull;
    }
#pragma unroll
    for (int j = 0; j < kSegCounters / kSegThreads; ++j) cnt[j * kSegThreads + tid] = 0;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSegItems; ++it) {
      const bool valid = it * kSegThreads + tid < n;
      const uint32_t d = (uint32_t)(x[it] >> shift) & mask;
      uint64_t peers = __ballot(valid);
      for (int b = 0; b < bits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t mb = __ballot(bit);
        peers &= bit ? mb : ~mb;
      }
      rk[it] = (uint32_t)__popcll(peers & lt);
      if (valid && (peers & lt) == 0)
        cnt[(d * kSegItems + it) * kSegWaves + wave] = (uint16_t)__popcll(peers);
    }
    __syncthreads();
    {  // exclusive scan of the counters, kSegCounters / kSegThreads per thread
      constexpr int kPer = kSegCounters / kSegThreads;
      uint32_t c[kPer], t = 0;
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        c[j] = cnt[kPer * tid + j];
        t += c[j];
      }
      uint32_t incl = t;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
      }
      if (lane == 63) s_part[wave] = incl;
      __syncthreads();
      uint32_t run = incl - t;
      for (int w = 0; w < wave; ++w) run += s_part[w];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        cnt[kPer * tid + j] = (uint16_t)run;
        run += c[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSegItems; ++it) {
      if (it * kSegThreads + tid < n) {
        const uint32_t d = (uint32_t)(x[it] >> shift) & mask;
        v[cnt[(d * kSegItems + it) * kSegWaves + wave] + rk[it]] = x[it];
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += kSegThreads) {
    const uint64_t y = v[i];
    kout[sg.r0 + i] = sg.base + (y >> kSegPosBits);
    iout[sg.r0 + i] = iin[sg.r0 + (int64_t)(y & (kSegCap - 1))];
  }
}

// starts[b] = first row of bucket b (rows sorted by their top bits), for
// the buckets that hold rows; the others keep -1.
__global__ __launch_bounds__(kBlock) void k_bucket_starts(const uint64_t* __restrict__ keys,
                                                          int64_t n, int low_bits,
                                                          int64_t* __restrict__ starts) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint64_t b = keys[i] >> low_bits;
  if (i == 0 || (keys[i - 1] >> low_bits) != b) starts[b] = i;
}

// Top bits B of the segmented sort for n > kSegCap rows of `bits`-bit keys
// (about 2,048 rows per bucket on average), or 0 where the plain LSD sort
// is used.
static int seg_bucket_bits(int64_t n, int bits) {
  if (n <= kSegCap || bits < 16) return 0;
  int B = 1;
  while (B < 16 && ((int64_t)2048 << B) < n) ++B;
  if (B < bits - kSegMaxKeyBits + 4) return 0;  // segments could span too few buckets
  return B;
}

uint64_t seg_sort_bytes(int64_t n, int bits) {
  const int B = seg_bucket_bits(n, bits);
  if (!B) return 0;
  return ((1ull << B) + 1) * (sizeof(int64_t) + sizeof(SortSeg)) + 256;
}

int sort_rows(uint64_t* ka, uint32_t* ia, uint64_t* kb, uint32_t* ib, int64_t n, int bits,
              uint32_t* tmp, void* scratch, hipStream_t s, int* which) {
  if (n > 1 && n <= kSegCap && bits <= kSegMaxKeyBits) {  // one segment: one launch
    const SortSeg one{0, (int32_t)n, bits, 0ull};
    hipLaunchKernelGGL(k_seg_sort, dim3(1), dim3(kSegThreads), 0, s, ka, ia, kb, ib,
                       (const SortSeg*)nullptr, one);
    *which = 1;
    return hipGetLastError() == hipSuccess ? 0 : 1;
  }
  const int B = seg_bucket_bits(n, bits);
  if (!B || !scratch) {
    *which = radix_sort(ka, ia, kb, ib, n, 1, bits, tmp, s);
    return 0;
  }
  const int low = bits - B;
  // ---- stable LSD passes over bits [low, bits): rows in bucket order
  int cur = 0;
  for (int shift = low; shift < bits; shift += 8) {
    const int w = (shift == low && B % 8) ? B % 8 : 8;
    if (cur == 0) sort_pass<1>(ka, ia, kb, ib, n, 0, shift, w, tmp, s);
    else sort_pass<1>(kb, ib, ka, ia, n, 0, shift, w, tmp, s);
    cur ^= 1;
    if (w != 8) shift -= 8 - w;
  }
  uint64_t* kx = cur ? kb : ka;  // bucket order
  uint32_t* ix = cur ? ib : ia;
  uint64_t* ky = cur ? ka : kb;  // result
  uint32_t* iy = cur ? ia : ib;
  // ---- bucket starts
  const uint64_t nbk = 1ull << B;
  int64_t* starts = static_cast<int64_t*>(scratch);
  SortSeg* dsegs = reinterpret_cast<SortSeg*>(starts + nbk + 1);
  launch_fill_u64(reinterpret_cast<uint64_t*>(starts), nbk, ~0ull, s);
  hipLaunchKernelGGL(k_bucket_starts, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, kx, n, low, starts);
  std::vector<int64_t> st(nbk + 1);
  if (hipMemcpyAsync(st.data(), starts, nbk * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return 1;
  st[nbk] = n;
  for (int64_t b = (int64_t)nbk - 1; b >= 0; --b)
    if (st[b] < 0) st[b] = st[b + 1];  // an empty bucket starts where the next does
  // ---- segments: runs of buckets within kSegCap rows whose key offsets fit
  std::vector<SortSeg> segs;
  std::vector<std::pair<int64_t, int64_t>> big;  // buckets sorted by the LSD passes
  const int span_bits = kSegMaxKeyBits - low;     // buckets per segment: 2^span_bits
  int64_t b0 = -1, last = -1, r0 = 0, cnt = 0;
  auto close = [&]() {
    if (cnt > 0) {
      const uint64_t rel_max = ((uint64_t)(last - b0 + 1) << low) - 1;
      const int nb = 64 - __builtin_clzll(rel_max);
      segs.push_back(SortSeg{r0, (int32_t)cnt, nb, (uint64_t)b0 << low});
    }
    cnt = 0;
    b0 = -1;
  };
  for (uint64_t b = 0; b < nbk; ++b) {
    const int64_t c = st[b + 1] - st[b];
    if (c == 0) continue;
    if (c > kSegCap) {
      close();
      big.emplace_back(st[b], c);
      continue;
    }
    if (cnt + c > kSegCap || (b0 >= 0 && ((int64_t)b - b0) >= (1ll << span_bits))) close();
    if (b0 < 0) {
      b0 = (int64_t)b;
      r0 = st[b];
    }
    last = (int64_t)b;
    cnt += c;
  }
  close();
  if (!segs.empty()) {
    if (hipMemcpyAsync(dsegs, segs.data(), segs.size() * sizeof(SortSeg),
                       hipMemcpyHostToDevice, s) != hipSuccess)
      return 1;
    hipLaunchKernelGGL(k_seg_sort, dim3((unsigned)segs.size()), dim3(kSegThreads), 0, s, kx,
                       ix, ky, iy, (const SortSeg*)dsegs, SortSeg{});
  }
  for (auto& bg : big) {  // rows of one bucket share its top bits
    const int w = radix_sort(kx + bg.first, ix + bg.first, ky + bg.first, iy + bg.first,
                             bg.second, 1, low, tmp, s);
    if (w == 0) {
      if (hipMemcpyAsync(ky + bg.first, kx + bg.first, bg.second * 8, hipMemcpyDeviceToDevice,
                         s) != hipSuccess ||
          hipMemcpyAsync(iy + bg.first, ix + bg.first, bg.second * 4, hipMemcpyDeviceToDevice,
                         s) != hipSuccess)
        return 1;
    }
  }
  // the segment table (host) must outlive its upload
  if (hipStreamSynchronize(s) != hipSuccess) return 1;
  *which = cur ? 0 : 1;
  return 0;
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
