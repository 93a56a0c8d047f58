// k-mer analysis kernels for gfx950: pack, window passes (Bloom pass A,
// counting pass B), classify + compact, gather.
//
// The window pass is the hot loop of the method (Section II-B: every read is
// cut into k-mers overlapping by k-1 bases, each occurrence updates the
// k-mer's count and its left/right extension tallies).  A block stages one
// tile of packed bases and bit planes in LDS, each lane forms the forward and
// reverse-complement words of its window from the staged tile, picks the
// canonical one, and updates an open-addressing table in HBM with 64-bit CAS
// (claim) and relaxed device-scope atomic adds (count and tallies).  The
// table's final contents do not depend on update order (Section II-A, Use
// case 1), which is what makes the unordered atomic updates exact.
#include "kh_internal.hpp"

namespace kh {

// ---------------------------------------------------------------- fill ----

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += stride)
    p[i] = v;
}

// Zero the per-count counters; keep only the status bits in `keep`.
__global__ void k_reset_ctr(unsigned long long* ctr, unsigned long long keep) {
  const int i = threadIdx.x;
  if (i < kCtrCount) ctr[i] = (i == kCtrStatus) ? (ctr[i] & keep) : 0ull;
}

void launch_reset_ctr(unsigned long long* ctr, uint64_t keep, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_ctr, dim3(1), dim3(64), 0, s, ctr,
                     (unsigned long long)keep);
}

void launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return;
  uint64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                     p, n, v);
}

// ---------------------------------------------------------------- pack ----

// One thread per 64 bases: ASCII bases and qualities -> 2-bit codes (two
// words), high-quality bits and non-base bits (one word each).
__global__ __launch_bounds__(kBlock) void k_pack(
    const uint8_t* __restrict__ seq, const uint8_t* __restrict__ qual,
    int64_t n, int qual_offset, int qual_cutoff, uint64_t* __restrict__ bases,
    uint64_t* __restrict__ hq, uint64_t* __restrict__ bad, int aligned) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t p0 = c * 64;
  if (p0 >= n) return;
  const int len = (n - p0) >= 64 ? 64 : (int)(n - p0);
  uint8_t sb[64], qb[64];
  if (aligned && len == 64) {
    const uint4* s4 = reinterpret_cast<const uint4*>(seq + p0);
    const uint4* q4 = reinterpret_cast<const uint4*>(qual + p0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      *reinterpret_cast<uint4*>(sb + 16 * i) = s4[i];
      *reinterpret_cast<uint4*>(qb + 16 * i) = q4[i];
    }
  } else {
    for (int i = 0; i < 64; ++i) {
      sb[i] = i < len ? seq[p0 + i] : (uint8_t)'N';
      qb[i] = i < len ? qual[p0 + i] : (uint8_t)0;
    }
  }
  uint64_t b0 = 0, b1 = 0, h = 0, x = 0;
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    const uint32_t ch = sb[i];
    const uint32_t up = ch & 0xDFu;  // fold lowercase
    const bool ok = (up == 'A') | (up == 'C') | (up == 'G') | (up == 'T');
    const uint64_t code = ((ch >> 1) ^ (ch >> 2)) & 3u;  // A0 C1 G2 T3, any case
    const bool good = ok && ((int)qb[i] - qual_offset >= qual_cutoff);
    if (i < 32) b0 |= code << (62 - 2 * i);
    else b1 |= code << (62 - 2 * (i - 32));
    h |= (uint64_t)good << (63 - i);
    x |= (uint64_t)(!ok) << (63 - i);
  }
  bases[2 * c] = b0;
  bases[2 * c + 1] = b1;
  hq[c] = h;
  bad[c] = x;
}

// One thread per read: mark its first base in the read-start plane and check
// the offsets (non-decreasing, offsets[0] == 0, offsets[n_reads] == n).
__global__ void k_mark_starts(const int64_t* __restrict__ off, int64_t n_reads,
                              int64_t n, uint64_t* __restrict__ st,
                              unsigned long long* __restrict__ ctr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > n_reads) return;
  const int64_t a = off[r];
  bool badoff = (r == 0 && a != 0) || (r == n_reads && a != n) || a < 0 || a > n;
  if (r < n_reads) {
    const int64_t b = off[r + 1];
    badoff |= b < a;
    if (!badoff && a < n && b > a)
      atomicOr(reinterpret_cast<unsigned long long*>(&st[a >> 6]),
               1ull << (63 - (a & 63)));
  }
  if (badoff) atomicOr(&ctr[kCtrStatus], (unsigned long long)kStatusBadOffsets);
}

void launch_pack(const PackArgs& a, hipStream_t s) {
  const int64_t chunks = (a.n + 63) / 64;
  if (chunks > 0) {
    const int aligned =
        ((reinterpret_cast<uintptr_t>(a.seq) | reinterpret_cast<uintptr_t>(a.qual)) & 15) == 0;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((chunks + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, a.seq, a.qual, a.n, a.qual_offset,
                       a.qual_cutoff, a.bases, a.hq, a.bad, aligned);
  }
  launch_fill_u64(a.st, (uint64_t)a.plane_words, 0ull, s);
  const int64_t threads = a.n_reads + 1;
  hipLaunchKernelGGL(k_mark_starts, dim3((unsigned)((threads + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, a.offsets, a.n_reads, a.n, a.st, a.ctr);
}

// ------------------------------------------------------- window passes ----

// Find the slot of `ch` (ws stored chunks) or claim one.  Each stored word is
// written once, by CAS from 0; a lane compares the words of a slot in order
// and, on meeting an empty word, CASes its own chunk in.  The words of a slot
// therefore always spell one inserted key, and lanes with equal keys stop at
// the same slot.  Returns nullptr if no slot was found within max_probe.
template <int C>
__device__ __forceinline__ uint8_t* find_or_claim(uint8_t* __restrict__ table,
                                                  uint64_t cap, uint32_t stride,
                                                  const uint64_t (&ch)[C],
                                                  int ws, uint64_t h,
                                                  uint32_t max_probe,
                                                  uint32_t& claimed) {
  uint64_t i = __umul64hi(h, cap);
  for (uint32_t probe = 0; probe < max_probe; ++probe) {
    uint64_t* s = reinterpret_cast<uint64_t*>(table + i * stride);
    bool match = true;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (c < ws && match) {
        uint64_t v = s[c];
        if (v == 0) {
          uint64_t expected = 0;
          if (__hip_atomic_compare_exchange_strong(
                  &s[c], &expected, ch[c], __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                  __HIP_MEMORY_SCOPE_AGENT)) {
            v = ch[c];
            if (c == 0) claimed++;
          } else {
            v = expected;
          }
        }
        match = (v == ch[c]);
      }
    }
    if (match) return reinterpret_cast<uint8_t*>(s);
    if (++i == cap) i = 0;
  }
  return nullptr;
}

// Bloom block of a key: two 64-bit words (level 1, level 2) and a pattern of
// up to four bits, from a hash independent of the table position.
__device__ __forceinline__ void bloom_slot(uint64_t h, uint64_t nblocks,
                                           uint64_t& blk, uint64_t& pat) {
  const uint64_t h2 = fmix64(h ^ 0xd6e8feb86659fd93ull);
  blk = __umul64hi(h2, nblocks);
  pat = (1ull << (h2 & 63)) | (1ull << ((h2 >> 6) & 63)) |
        (1ull << ((h2 >> 12) & 63)) | (1ull << ((h2 >> 18) & 63));
}

// MODE 0: count every window.  MODE 1: Bloom pass A (record sightings).
// MODE 2: count the windows whose key passed level 2 of the Bloom filter.
// MODE 3: heavy-hitter recount -- exact 32-bit extension tallies for the
//         k-mers listed in the heavy index (the main table is not touched).
template <int W, int MODE>
__global__ __launch_bounds__(kBlock) void k_windows(WindowArgs a) {
  __shared__ uint64_t s_bases[kBaseWords];
  __shared__ uint64_t s_hq[kPlaneWords];
  __shared__ uint64_t s_bad[kPlaneWords];
  __shared__ uint64_t s_st[kPlaneWords];
  __shared__ uint64_t s_red[kBlock / 64];

  const int64_t P0 = (int64_t)blockIdx.x * kTile;
  const int64_t O = P0 - kHalo;  // staged origin, a multiple of 64
  const int tid = threadIdx.x;
  for (int i = tid; i < kBaseWords; i += kBlock) {
    const int64_t gw = O / 32 + i;
    s_bases[i] = (gw >= 0 && gw < a.base_words) ? a.bases[gw] : 0ull;
  }
  for (int i = tid; i < kPlaneWords; i += kBlock) {
    const int64_t gw = O / 64 + i;
    const bool in = gw >= 0 && gw < a.plane_words;
    s_hq[i] = in ? a.hq[gw] : 0ull;
    s_bad[i] = in ? a.bad[gw] : ~0ull;
    s_st[i] = in ? a.st[gw] : 0ull;
  }
  __syncthreads();

  const uint32_t k = a.k;
  const int ws = table_chunks(k);
  const SlotLayout lay = slot_layout(ws);
  uint64_t n_win = 0, n_l1 = 0, n_l2 = 0;
  uint32_t n_claim = 0;
  bool fail = false;

  for (int j = 0; j < kTile / kBlock; ++j) {
    const int64_t p = P0 + j * kBlock + tid;
    if (p + (int64_t)k > a.n) continue;
    const uint32_t lp = (uint32_t)(p - O);
    if (any_bits(s_bad, lp, k) || any_bits(s_st, lp + 1, k - 1)) continue;
    ++n_win;

    uint64_t f[W], r[W], key[W];
    window_words<W>(s_bases, 2 * lp, k, f);
    revcomp_words<W>(f, k, r);
    const bool use_rc = words_less<W>(r, f);
#pragma unroll
    for (int w = 0; w < W; ++w) key[w] = use_rc ? r[w] : f[w];
    uint64_t ch[W + 1];
    to_chunks<W, W + 1>(key, ws, ch);
    const uint64_t h = hash_chunks<W + 1>(ch, ws);

    if (MODE == 1) {
      uint64_t blk, pat;
      bloom_slot(h, a.bloom_blocks, blk, pat);
      uint64_t* b = a.bloom + 2 * blk;
      const uint64_t old1 = __hip_atomic_fetch_or(&b[0], pat, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
      if ((old1 & pat) != pat) {
        ++n_l1;
      } else if ((b[1] & pat) != pat) {
        const uint64_t old2 = __hip_atomic_fetch_or(
            &b[1], pat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((old2 & pat) != pat) ++n_l2;
      }
      continue;
    }
    if (MODE == 2) {
      uint64_t blk, pat;
      bloom_slot(h, a.bloom_blocks, blk, pat);
      if ((a.bloom[2 * blk + 1] & pat) != pat) continue;
    }
    HeavyEntry* he = nullptr;
    if (MODE == 3) {
      uint32_t x = (uint32_t)(h >> 32) & a.heavy_mask;
      for (uint32_t probe = 0; probe <= a.heavy_mask; ++probe) {
        const uint32_t e = a.heavy_index[x];
        if (e == kHeavyEmpty) break;
        bool eq = true;
#pragma unroll
        for (int c = 0; c < W + 1; ++c)
          if (c < ws) eq = eq && (a.heavy[e].chunks[c] == ch[c]);
        if (eq) {
          he = &a.heavy[e];
          break;
        }
        x = (x + 1) & a.heavy_mask;
      }
      if (!he) continue;
    }

    // extensions seen from the read's strand
    int L = -1, R = -1;
    if (!get_bit(s_st, lp) && get_bit(s_hq, lp - 1)) L = (int)get_base(s_bases, lp - 1);
    if (p + (int64_t)k < a.n && !get_bit(s_st, lp + k) && get_bit(s_hq, lp + k))
      R = (int)get_base(s_bases, lp + k);
    if (use_rc) {  // other strand: sides swap, bases complement
      const int t = L;
      L = R >= 0 ? 3 - R : -1;
      R = t >= 0 ? 3 - t : -1;
    }

    if (MODE == 3) {
      if (L >= 0) atomicAdd(&he->ext[L], 1u);
      if (R >= 0) atomicAdd(&he->ext[4 + R], 1u);
      continue;
    }
    uint8_t* s = find_or_claim<W + 1>(a.table, a.capacity, lay.stride, ch, ws,
                                      h, a.max_probe, n_claim);
    if (!s) {
      fail = true;
      continue;
    }
    __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(s + lay.count_off), 1u,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (L >= 0)
      __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(s + lay.left_off),
                             1ull << (16 * L), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    if (R >= 0)
      __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(s + lay.right_off),
                             1ull << (16 * R), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }

  if (MODE == 3) return;
  if (fail) atomicOr(&a.ctr[kCtrStatus], (unsigned long long)kStatusProbeLimit);
  if (MODE == 1) {
    block_add(&a.ctr[kCtrL1New], n_l1, s_red);
    __syncthreads();
    block_add(&a.ctr[kCtrL2New], n_l2, s_red);
  } else {
    block_add(&a.ctr[kCtrClaimed], n_claim, s_red);
  }
  __syncthreads();
  if (MODE != 2 || a.count_windows) block_add(&a.ctr[kCtrWindows], n_win, s_red);
}

template <int W>
static void launch_windows_w(const WindowArgs& a, int mode, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.n + kTile - 1) / kTile);
  if (blocks == 0) return;
  if (mode == 0)
    hipLaunchKernelGGL((k_windows<W, 0>), dim3(blocks), dim3(kBlock), 0, s, a);
  else if (mode == 1)
    hipLaunchKernelGGL((k_windows<W, 1>), dim3(blocks), dim3(kBlock), 0, s, a);
  else if (mode == 2)
    hipLaunchKernelGGL((k_windows<W, 2>), dim3(blocks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_windows<W, 3>), dim3(blocks), dim3(kBlock), 0, s, a);
}

void launch_windows(const WindowArgs& a, int mode, hipStream_t s) {
  switch ((a.k + 31) / 32) {
    case 1: launch_windows_w<1>(a, mode, s); break;
    case 2: launch_windows_w<2>(a, mode, s); break;
    case 3: launch_windows_w<3>(a, mode, s); break;
    default: launch_windows_w<4>(a, mode, s); break;
  }
}

// ----------------------------------------------------- classify/compact ----

// Keep occupied slots with count >= min_count: write their key in export
// words and their slot index, at positions taken with one atomic per wave.
template <int W>
__global__ __launch_bounds__(kBlock) void k_classify(ClassifyArgs a) {
  const int ws = table_chunks(a.k);
  const SlotLayout lay = slot_layout(ws);
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < a.capacity;
       base += stride) {
    const uint64_t i = base + threadIdx.x;
    bool keep = false;
    const uint8_t* s = a.table + i * lay.stride;
    uint32_t cnt = 0;
    if (i < a.capacity) {
      const uint64_t c0 = *reinterpret_cast<const uint64_t*>(s);
      cnt = *reinterpret_cast<const uint32_t*>(s + lay.count_off);
      keep = c0 != 0 && cnt >= a.min_count;
    }
    const uint64_t pos = wave_append(&a.ctr[kCtrRows], keep);
    if (keep) {
      if (cnt > 65535u) {  // 16-bit tallies may have wrapped: recount later
        atomicOr(&a.ctr[kCtrStatus], (unsigned long long)kStatusHeavy);
        const uint64_t hp = atomicAdd(&a.ctr[kCtrHeavy], 1ull);
        if (hp < kHeavyMax) a.heavy_list[hp] = (uint32_t)i;
      }
      uint64_t f[W];
      from_chunks<W>(reinterpret_cast<const uint64_t*>(s), ws, f);
#pragma unroll
      for (int w = 0; w < W; ++w) a.keys_out[pos * W + w] = f[w];
      a.idx_out[pos] = (uint32_t)i;
    }
  }
}

void launch_classify(const ClassifyArgs& a, hipStream_t s) {
  if (a.capacity == 0) return;
  uint64_t blocks = (a.capacity + kBlock - 1) / kBlock;
  if (blocks > 16384) blocks = 16384;
  switch ((a.k + 31) / 32) {
    case 1: hipLaunchKernelGGL(k_classify<1>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_classify<2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_classify<3>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
    default: hipLaunchKernelGGL(k_classify<4>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
  }
}

// --------------------------------------------------------- heavy build ----

// One thread per heavy k-mer: copy its stored key into a heavy entry, index
// the entry by hash, and leave the entry number in the slot's left tally word
// (the 16-bit tallies of a heavy slot are no longer used).
__global__ void k_heavy_build(HeavyBuildArgs a) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.n_heavy) return;
  const int ws = table_chunks(a.k);
  const SlotLayout lay = slot_layout(ws);
  uint8_t* s = a.table + (uint64_t)a.heavy_list[h] * lay.stride;
  const uint64_t* sc = reinterpret_cast<const uint64_t*>(s);
  HeavyEntry& e = a.heavy[h];
  uint64_t c[5];
  for (int j = 0; j < 5; ++j) c[j] = j < ws ? sc[j] : 0ull;
  for (int j = 0; j < 5; ++j) e.chunks[j] = c[j];
  e.slot = a.heavy_list[h];
  e.pad = 0;
  for (int j = 0; j < 8; ++j) e.ext[j] = 0;
  uint64_t hh = 0x9e3779b97f4a7c15ull;
  for (int j = 0; j < ws; ++j) hh = fmix64(hh ^ c[j]);
  uint32_t x = (uint32_t)(hh >> 32) & a.heavy_mask;
  for (uint32_t probe = 0; probe <= a.heavy_mask; ++probe) {
    if (atomicCAS(&a.heavy_index[x], kHeavyEmpty, h) == kHeavyEmpty) break;
    x = (x + 1) & a.heavy_mask;
  }
  *reinterpret_cast<uint64_t*>(s + lay.left_off) = (uint64_t)h;
}

void launch_heavy_build(const HeavyBuildArgs& a, hipStream_t s) {
  if (a.n_heavy == 0) return;
  hipLaunchKernelGGL(k_heavy_build, dim3((a.n_heavy + kBlock - 1) / kBlock),
                     dim3(kBlock), 0, s, a);
}

// ------------------------------------------------------------- gather ----

// Extension letter of one side (tallies c, depth d): dead end 'X' if the most
// common base is seen fewer than t_min_ext times, fork 'F' on a tie or when
// more than t_hq = max(t_base, e*d) observations contradict it (Section
// II-C's depth-adaptive rule, e = err_ppm / 10^6, compared in integers).
__device__ __forceinline__ uint8_t side_code(const uint32_t (&c)[4], uint64_t d,
                                             uint32_t t_min_ext, uint32_t t_base,
                                             uint32_t err_ppm) {
  uint32_t m = c[0];
  int best = 0;
#pragma unroll
  for (int b = 1; b < 4; ++b)
    if (c[b] > m) { m = c[b]; best = b; }
  if (m < t_min_ext) return 'X';
  const int ties = (c[0] == m) + (c[1] == m) + (c[2] == m) + (c[3] == m);
  if (ties > 1) return 'F';
  const uint64_t alt = (uint64_t)c[0] + c[1] + c[2] + c[3] - m;
  const uint64_t lim_a = (uint64_t)t_base * 1000000ull;
  const uint64_t lim_b = (uint64_t)err_ppm * d;
  const uint64_t lim = lim_a > lim_b ? lim_a : lim_b;
  const uint8_t letters[4] = {'A', 'C', 'G', 'T'};
  return alt * 1000000ull <= lim ? letters[best] : (uint8_t)'F';
}

__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs a) {
  const int ws = table_chunks(a.k);
  const SlotLayout lay = slot_layout(ws);
  const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (row >= a.n_rows) return;
  const uint8_t* s = a.table + (uint64_t)a.idx[row] * lay.stride;
  const uint32_t cnt = *reinterpret_cast<const uint32_t*>(s + lay.count_off);
  const uint64_t lw = *reinterpret_cast<const uint64_t*>(s + lay.left_off);
  const uint64_t rw = *reinterpret_cast<const uint64_t*>(s + lay.right_off);
  uint32_t l[4], r[4];
  if (cnt > 65535u) {  // heavy hitter: exact tallies from the recount
    const HeavyEntry& e = a.heavy[lw];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      l[b] = e.ext[b];
      r[b] = e.ext[4 + b];
    }
  } else {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      l[b] = (uint32_t)((lw >> (16 * b)) & 0xffffu);
      r[b] = (uint32_t)((rw >> (16 * b)) & 0xffffu);
    }
  }
  a.counts[row] = cnt;
  uint4* e = reinterpret_cast<uint4*>(a.ext + row * 8);
  e[0] = make_uint4(l[0], l[1], l[2], l[3]);
  e[1] = make_uint4(r[0], r[1], r[2], r[3]);
  a.codes[2 * row] = side_code(l, cnt, a.t_min_ext, a.t_base, a.err_ppm);
  a.codes[2 * row + 1] = side_code(r, cnt, a.t_min_ext, a.t_base, a.err_ppm);
}

void launch_gather(const GatherArgs& a, hipStream_t s) {
  if (a.n_rows == 0) return;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((a.n_rows + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, a);
}

}  // namespace kh
