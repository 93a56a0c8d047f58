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

void launch_pack_range(const PackArgs& a, int64_t p0, int64_t p1, hipStream_t s) {
  const int64_t chunks = (p1 - p0 + 63) / 64;
  if (chunks <= 0) return;
  const uint8_t* seq = a.seq + p0;
  const uint8_t* qual = a.qual + p0;
  const int aligned =
      ((reinterpret_cast<uintptr_t>(seq) | reinterpret_cast<uintptr_t>(qual)) & 15) == 0;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((chunks + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, seq, qual, p1 - p0, a.qual_offset,
                     a.qual_cutoff, a.bases + p0 / 32, a.hq + p0 / 64, a.bad + p0 / 64,
                     aligned);
}

void launch_pack(const PackArgs& a, hipStream_t s) {
  launch_pack_range(a, 0, a.n, s);
  launch_mark_starts(a, s);
}

void launch_mark_starts(const PackArgs& a, hipStream_t s) {
  launch_fill_u64(a.st, (uint64_t)a.plane_words, 0ull, s);
  const int64_t threads = a.n_reads + 1;
  hipLaunchKernelGGL(k_mark_starts, dim3((unsigned)((threads + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, a.offsets, a.n_reads, a.n, a.st, a.ctr);
}

// ------------------------------------------------------- window passes ----

// Find the slot of `ch` (ws stored chunks) or claim one, starting at slot i
// whose stored words `w0` the caller has already loaded.  Each stored word
// is written once, by CAS from 0; a lane compares the words of a slot in
// order and, on meeting an empty word, CASes its own chunk in.  The words of
// a slot therefore always spell one inserted key, and lanes with equal keys
// stop at the same slot.  All words of a slot are loaded at once (one round
// trip, not one per word): a word read as 0 may have been written since,
// which the CAS then reports, and a non-zero word is final.  Returns nullptr
// if no slot was found within max_probe slots.
// The first ws stored words of a slot (the rest 0), loaded together.
template <int C>
__device__ __forceinline__ void load_slot_words(const uint8_t* slot, int ws, uint64_t (&w)[C]) {
  const uint64_t* p = reinterpret_cast<const uint64_t*>(slot);
#pragma unroll
  for (int c = 0; c < C; ++c) w[c] = c < ws ? p[c] : 0ull;
}

template <int C>
__device__ __forceinline__ uint8_t* find_or_claim(uint8_t* __restrict__ table,
                                                  uint64_t cap, uint32_t stride,
                                                  const uint64_t (&ch)[C],
                                                  int ws, uint64_t i, const uint64_t (&w0)[C],
                                                  uint32_t max_probe,
                                                  uint32_t& claimed) {
  for (uint32_t probe = 0; probe < max_probe; ++probe) {
    uint64_t* s = reinterpret_cast<uint64_t*>(table + i * stride);
    uint64_t w[C];
    if (probe == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) w[c] = w0[c];
    } else {
      load_slot_words<C>(reinterpret_cast<const uint8_t*>(s), ws, w);
    }
    bool match = true;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (c < ws && match) {
        uint64_t v = w[c];
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

// Bloom word of a key and its pattern of up to four bits within a 32-bit
// half, from a hash independent of the table position.  Level 1 ("seen")
// uses the low half of the word, level 2 ("seen twice") the high half, so
// one returning atomicOr both records a sighting and reports both levels.
__device__ __forceinline__ void bloom_slot(uint64_t h, uint64_t nwords,
                                           uint64_t& blk, uint32_t& pat) {
  const uint64_t h2 = fmix64(h ^ 0xd6e8feb86659fd93ull);
  blk = __umul64hi(h2, nwords);
  pat = (1u << (h2 & 31)) | (1u << ((h2 >> 5) & 31)) |
        (1u << ((h2 >> 10) & 31)) | (1u << ((h2 >> 15) & 31));
}

// MODE 0: count every window.  MODE 1: Bloom pass A (record sightings).
// MODE 2: count the windows whose key passed level 2 of the Bloom filter.
// MODE 3: heavy-hitter recount -- exact 32-bit count and extension tallies
//         for the k-mers listed in the heavy index (the table is untouched).
//
// A sub-pass gives each lane J windows of the staged tile (J = 1, 2 or 4;
// kTile / (J * kBlock) sub-passes cover the tile).  All J are formed first
// (LDS + ALU only); then each memory step is issued for every window before
// any result is consumed, so a lane keeps J random accesses in flight
// instead of waiting out one round trip per window.  Larger J hides more
// latency, smaller J needs fewer registers (more waves per SIMD): the best
// J depends on the key width and the pass, and is a tuning parameter.

// Per-thread tallies of a block's sub-passes, added to the global counters
// once per block so that few atomics hit the counters' addresses.
struct PassCounts {
  uint32_t win = 0, l1 = 0, l2 = 0, pass = 0, claim = 0;
  bool fail = false;
};

// One sub-pass of one staged tile for one k: form windows w0 + j * kBlock +
// tid (j < J) of the tile starting at P0, then run the pass (MODE) over
// them.  Called by the single-k kernel and by the fused multi-k Bloom
// kernel; all threads of the block call it together.  `tile_id` names the
// tile in overflow entries.
template <int W, int MODE, int J>
__device__ __forceinline__ void tile_pass(
    const uint64_t* s_bases, const uint64_t* s_hq, const uint64_t* s_bad,
    const uint64_t* s_st, int64_t P0, int64_t O, int w0, int64_t n_end,
    uint32_t k, uint64_t* bloom, uint64_t bloom_blocks, uint64_t* seen, uint8_t* table,
    uint64_t capacity, uint32_t max_probe, HeavyEntry* heavy,
    const uint32_t* heavy_index, uint32_t heavy_mask, PassCounts& pc,
    uint64_t* overflow, unsigned long long* overflow_n, uint64_t overflow_cap,
    uint64_t tile_id, int tid, uint32_t shards, uint32_t owner) {
  constexpr int C = W + 1;
  // Keep the compiler from hoisting this sub-pass's LDS addressing (which
  // depends only on tid, w0 and j) out of the caller's loops: held across
  // the loop it would take a register per address.
  asm volatile("" : "+v"(tid));
  const int ws = table_chunks(k);
  const SlotLayout lay = slot_layout(ws);

  // ---- form the windows: canonical key chunks, hash, extensions
  bool ok[J];
  uint64_t ch[J][C];
  uint64_t hh[J];
  int L[J], R[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    ok[j] = false;
    hh[j] = 0;
    L[j] = R[j] = -1;
#pragma unroll
    for (int c = 0; c < C; ++c) ch[j][c] = 0;
    const int64_t p = P0 + w0 + j * kBlock + tid;
    if (p + (int64_t)k > n_end) continue;
    const uint32_t lp = (uint32_t)(p - O);
    if (any_bits(s_bad, lp, k) || any_bits(s_st, lp + 1, k - 1)) continue;
    uint64_t f[W], r[W], key[W];
    window_words<W>(s_bases, 2 * lp, k, f);
    revcomp_words<W>(f, k, r);
    const bool use_rc = words_less<W>(r, f);
#pragma unroll
    for (int w = 0; w < W; ++w) key[w] = use_rc ? r[w] : f[w];
    if (shards > 1 && owner_of<W>(key, shards) != owner) continue;  // another part's key
    ok[j] = true;
    ++pc.win;
    to_chunks<W, C>(key, ws, ch[j]);
    hh[j] = hash_chunks<C>(ch[j], ws);
    if (MODE != 1) {  // extensions seen from the read's strand
      int l = -1, rr = -1;
      if (!get_bit(s_st, lp) && get_bit(s_hq, lp - 1)) l = (int)get_base(s_bases, lp - 1);
      if (p + (int64_t)k < n_end && !get_bit(s_st, lp + k) && get_bit(s_hq, lp + k))
        rr = (int)get_base(s_bases, lp + k);
      if (use_rc) {  // other strand: sides swap, bases complement
        L[j] = rr >= 0 ? 3 - rr : -1;
        R[j] = l >= 0 ? 3 - l : -1;
      } else {
        L[j] = l;
        R[j] = rr;
      }
    }
  }

  if (MODE == 1) {
    // ---- Bloom pass A: record every sighting; complete level 2 on a repeat.
    // A plain load comes first: a key whose level-2 pattern is already
    // complete (its third and later sightings, most windows at any useful
    // coverage) needs no atomic, and one whose level-1 pattern is complete
    // needs only the level-2 one.  Bits are only ever set, so whatever the
    // load returns (even a stale copy) is a subset of the word's final
    // bits: every decision it leads to is one the atomics would also allow.
    uint64_t blk[J], cur[J];
    uint32_t pat[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      cur[j] = 0;
      if (ok[j]) {
        bloom_slot(hh[j], bloom_blocks, blk[j], pat[j]);
        cur[j] = bloom[blk[j]];
      }
    }
    bool set1[J], set2[J];
    uint64_t old[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      set1[j] = ok[j] && ((uint32_t)cur[j] & pat[j]) != pat[j];
      set2[j] = ok[j] && !set1[j] && ((uint32_t)(cur[j] >> 32) & pat[j]) != pat[j];
      old[j] = 0;
      if (set1[j] || set2[j])
        old[j] = __hip_atomic_fetch_or(bloom + blk[j],
                                       set1[j] ? (uint64_t)pat[j] : (uint64_t)pat[j] << 32,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    bool second[J];
    uint64_t old2[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      second[j] = false;
      old2[j] = 0;
      if (set1[j]) {
        if (((uint32_t)old[j] & pat[j]) != pat[j]) {
          ++pc.l1;  // first sighting (up to false positives)
        } else if (((uint32_t)(old[j] >> 32) & pat[j]) != pat[j]) {
          second[j] = true;  // seen meanwhile: complete the level-2 pattern
          old2[j] = __hip_atomic_fetch_or(bloom + blk[j], (uint64_t)pat[j] << 32,
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      } else if (set2[j] && ((uint32_t)(old[j] >> 32) & pat[j]) != pat[j]) {
        ++pc.l2;  // this sighting completed level 2
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j)
      if (second[j] && ((uint32_t)(old2[j] >> 32) & pat[j]) != pat[j]) ++pc.l2;
    if (seen) {  // one word per wave: its 64 windows are consecutive positions
#pragma unroll
      for (int j = 0; j < J; ++j) {
        // level 1 was complete before this window (at the load, or by the
        // atomic's return): the key had been seen, so this window or an
        // earlier one completes level 2
        const bool again =
            ok[j] && (!set1[j] || ((uint32_t)old[j] & pat[j]) == pat[j]);
        const uint64_t m = __ballot(again);
        if ((tid & 63) == 0) seen[(P0 + w0 + j * kBlock + tid) >> 6] = m;
      }
    }
  } else if (MODE == 3) {
    // ---- heavy-hitter recount (rare): look up each window in the small index
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (!ok[j]) continue;
      HeavyEntry* he = nullptr;
      uint32_t x = (uint32_t)(hh[j] >> 32) & heavy_mask;
      for (uint32_t probe = 0; probe <= heavy_mask; ++probe) {
        const uint32_t e = heavy_index[x];
        if (e == kHeavyEmpty) break;
        bool eq = true;
#pragma unroll
        for (int c = 0; c < C; ++c)
          if (c < ws) eq = eq && (heavy[e].chunks[c] == ch[j][c]);
        if (eq) {
          he = &heavy[e];
          break;
        }
        x = (x + 1) & heavy_mask;
      }
      if (!he) continue;
      atomicAdd(&he->count, 1u);
      if (L[j] >= 0) atomicAdd(&he->ext[L[j]], 1u);
      if (R[j] >= 0) atomicAdd(&he->ext[4 + R[j]], 1u);
    }
    return;
  } else {
    // ---- counting pass
    if (MODE == 2) {  // keep the windows whose key completed Bloom level 2
      bool known[J];   // pass A saw this window's key before: level 2 complete
#pragma unroll
      for (int j = 0; j < J; ++j) {
        known[j] = false;
        if (seen) {
          const uint64_t m = seen[(P0 + w0 + j * kBlock + (tid & ~63)) >> 6];
          known[j] = (m >> (tid & 63)) & 1;
        }
      }
      uint64_t bw[J];
      uint32_t pat[J];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        bw[j] = 0;
        pat[j] = 0;
        if (ok[j] && !known[j]) {
          uint64_t blk;
          bloom_slot(hh[j], bloom_blocks, blk, pat[j]);
          bw[j] = bloom[blk];
        }
      }
#pragma unroll
      for (int j = 0; j < J; ++j)
        if (ok[j] && !known[j] && ((uint32_t)(bw[j] >> 32) & pat[j]) != pat[j]) ok[j] = false;
    }
    uint64_t slot0[J], word0[J][C];
#pragma unroll
    for (int j = 0; j < J; ++j) {  // first probe of every window at once
      slot0[j] = 0;
#pragma unroll
      for (int c = 0; c < C; ++c) word0[j][c] = 0;
      if (ok[j]) {
        slot0[j] = __umul64hi(hh[j], capacity);
        load_slot_words<C>(table + slot0[j] * lay.stride, ws, word0[j]);
      }
    }
    uint8_t* sp[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      sp[j] = nullptr;
      if (!ok[j]) continue;
      ++pc.pass;
      sp[j] = find_or_claim<C>(table, capacity, lay.stride, ch[j], ws,
                               slot0[j], word0[j], max_probe, pc.claim);
      if (!sp[j]) {
        if (overflow) {  // batched launch: keep the window for the replay
          const uint64_t e = atomicAdd(overflow_n, 1ull);
          if (e < overflow_cap)
            overflow[e] = (tile_id << 10) | (uint64_t)(w0 + j * kBlock + tid);
          else
            pc.fail = true;
        } else {
          pc.fail = true;
        }
      }
    }
    uint64_t oldx[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {  // one returning add: count + both tallies
      oldx[j] = 0;
      if (!sp[j]) continue;
      oldx[j] = __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(sp[j] + lay.x_off),
                                       x_increment(L[j], R[j]), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {  // spill occurrences also count exactly
      if (!sp[j]) continue;
      const uint32_t c = (uint32_t)(oldx[j] & kCountMask);
      if (c < kSpillAt) continue;
      if (L[j] >= 0)
        __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(sp[j] + lay.sl_off),
                               1ull << (16 * L[j]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      if (R[j] >= 0)
        __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(sp[j] + lay.sr_off),
                               1ull << (16 * R[j]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      if (c == kHeavyCount - 1)  // once per 2^16 occurrences: mark heavy
        __hip_atomic_fetch_or(reinterpret_cast<uint64_t*>(sp[j] + lay.sr_off),
                              kHeavyBit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }

}

// Add a block's tallies to the counters (all threads of the block call it).
template <int MODE>
__device__ __forceinline__ void flush_counts(const PassCounts& pc,
                                             unsigned long long* ctr,
                                             unsigned long long* tile_ctr,
                                             int count_windows, uint64_t* s_red) {
  if (MODE == 3) return;
  if (pc.fail) atomicOr(&ctr[kCtrStatus], (unsigned long long)kStatusProbeLimit);
  if (MODE == 1) {
    block_add(&ctr[kCtrL1New], pc.l1, s_red);
    __syncthreads();
    block_add(&ctr[kCtrL2New], pc.l2, s_red);
  } else if (tile_ctr) {  // batched launch: per read set and table
    block_add(&tile_ctr[0], pc.claim, s_red);
    __syncthreads();
    block_add(&tile_ctr[1], pc.win, s_red);
    return;
  } else {
    block_add(&ctr[kCtrClaimed], pc.claim, s_red);
    __syncthreads();
    block_add(&ctr[kCtrPassed], pc.pass, s_red);
  }
  __syncthreads();
  if (MODE != 2 || count_windows) block_add(&ctr[kCtrWindows], pc.win, s_red);
}

// Launch over one read set: block b takes tiles b, b + grid, ... (the grid
// is a tuning parameter) and adds its tallies once.  Batched launch (a.tiles
// set): one block per descriptor, which names the read set, range, table and
// counters of its tile.
template <int W, int MODE, int J>
__global__ __launch_bounds__(kBlock) void k_windows(WindowArgs a) {
  __shared__ uint64_t s_bases[kBaseWords];
  __shared__ uint64_t s_hq[kPlaneWords];
  __shared__ uint64_t s_bad[kPlaneWords];
  __shared__ uint64_t s_st[kPlaneWords];
  __shared__ uint64_t s_red[kBlock / 64];
  PassCounts pc;
  if (a.tiles) {
    const TileDesc& d = a.tiles[blockIdx.x];
    const int64_t O = d.p0 - kHalo;  // staged origin, a multiple of 64
    stage_tile(d.bases, d.hq, d.bad, d.st, d.base_words, d.plane_words, O, s_bases,
               s_hq, s_bad, s_st);
    __syncthreads();
    const uint32_t max_probe =
        d.overflow ? 1024u : (d.capacity < 0xffffffffull ? (uint32_t)d.capacity : 0xffffffffu);
    for (int w0 = 0; w0 < kTile; w0 += J * kBlock)
      tile_pass<W, MODE, J>(s_bases, s_hq, s_bad, s_st, d.p0, O, w0, d.hi, a.k, a.bloom,
                            a.bloom_blocks, nullptr, d.table, d.capacity, max_probe, d.heavy,
                            d.heavy_index, d.heavy_mask, pc, d.overflow, d.overflow_n,
                            d.overflow_cap, blockIdx.x, (int)threadIdx.x, 0u, 0u);
    flush_counts<MODE>(pc, a.ctr, d.counters, a.count_windows, s_red);
    return;
  }
  const int64_t n_tiles = a.t_end > 0 ? a.t_end : (a.n + kTile - 1) / kTile;
  for (int64_t t = a.t_begin + blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t P0 = t * kTile, O = P0 - kHalo;
    __syncthreads();  // every window of the previous tile is formed
    stage_tile(a.bases, a.hq, a.bad, a.st, a.base_words, a.plane_words, O, s_bases, s_hq,
               s_bad, s_st);
    __syncthreads();
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    for (int w0 = 0; w0 < kTile; w0 += J * kBlock)
      tile_pass<W, MODE, J>(s_bases, s_hq, s_bad, s_st, P0, O, w0, a.n, a.k, a.bloom,
                            a.bloom_blocks, a.seen, a.table, a.capacity, a.max_probe, a.heavy,
                            a.heavy_index, a.heavy_mask, pc, nullptr, nullptr, 0,
                            (uint64_t)t, tid, a.shards, a.owner);
  }
  flush_counts<MODE>(pc, a.ctr, nullptr, a.count_windows, s_red);
}

// ---------------------------------------------- aggregating counting pass ----
//
// Counting pass B for reads in an order that keeps a k-mer's occurrences
// close (minimizer order): a block takes `tiles_per_block` consecutive
// tiles; in each tile every window that passes the Bloom screen is merged
// into an LDS map keyed by its canonical k-mer (count and 16-bit tallies
// per base, summed with LDS atomics), then every distinct k-mer of the tile
// updates the table once.  The map stores, per entry, a 32-bit tag from the
// key's hash and the tile position of the window that claimed it; a window
// whose tag matches compares its key with the claimer's, re-formed from the
// staged tile, so no key is stored twice and nothing waits.  A window that
// finds no entry within kAggProbe probes updates the table directly.
//
// An aggregated update adds m occurrences in one returning add to the
// packed counter.  Of those, the ones at positions kSpillAt and beyond (from
// the returned count) are spill occurrences, whose tallies go to SL/SR as
// usual; which occurrences they are does not matter, only that the other
// ones carry at most one tally per occurrence per side, so the spill part
// takes at least (tallies - non-spill occurrences) of each side's tallies.
// The packed fields of the non-spill occurrences then sum to at most
// kSpillAt in all, and decode_slot stays exact.

constexpr int kAggSlots = 1024;  // one tile's windows at most
constexpr int kAggProbe = 32;

// Canonical key chunks, hash and use_rc of the window at staged position lp.
template <int W, int C>
__device__ __forceinline__ void staged_key(const uint64_t* s_bases, uint32_t lp, uint32_t k,
                                           int ws, uint64_t (&ch)[C], uint64_t& h,
                                           bool& use_rc) {
  uint64_t f[W], r[W], key[W];
  window_words<W>(s_bases, 2 * lp, k, f);
  revcomp_words<W>(f, k, r);
  use_rc = words_less<W>(r, f);
#pragma unroll
  for (int w = 0; w < W; ++w) key[w] = use_rc ? r[w] : f[w];
#pragma unroll
  for (int c = 0; c < C; ++c) ch[c] = 0;
  to_chunks<W, C>(key, ws, ch);
  h = hash_chunks<C>(ch, ws);
}

// Table update for m occurrences of one k-mer with left/right tallies l, r
// (l[b], r[b] count the occurrences whose extension is base b).
template <int C>
__device__ __forceinline__ void agg_update(uint8_t* sp, const SlotLayout& lay, uint32_t m,
                                           const uint32_t (&l)[4], const uint32_t (&r)[4]) {
  uint64_t inc = m;
  uint32_t sl = 0, sr = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    inc += (uint64_t)l[b] << (16 + 6 * b);
    inc += (uint64_t)r[b] << (40 + 6 * b);
    sl += l[b];
    sr += r[b];
  }
  const uint64_t old = __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(sp + lay.x_off), inc,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t c = (uint32_t)(old & kCountMask);
  const uint32_t keep = c < kSpillAt ? min(m, kSpillAt - c) : 0u;  // non-spill occurrences
  if (keep < m) {
    // spill tallies: at least (tallies - keep) per side, taken base by base
    uint32_t need_l = sl > keep ? sl - keep : 0u, need_r = sr > keep ? sr - keep : 0u;
    uint64_t add_l = 0, add_r = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t tl = min(l[b], need_l), tr = min(r[b], need_r);
      need_l -= tl;
      need_r -= tr;
      add_l += (uint64_t)tl << (16 * b);
      add_r += (uint64_t)tr << (16 * b);
    }
    if (add_l)
      __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(sp + lay.sl_off), add_l,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (add_r)
      __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(sp + lay.sr_off), add_r,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // an occurrence at count kHeavyCount - 1 (mod 2^16) marks the k-mer heavy
  if (((kHeavyCount - 1u - c) & 0xffffu) < m)
    __hip_atomic_fetch_or(reinterpret_cast<uint64_t*>(sp + lay.sr_off), kHeavyBit,
                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_count_agg(WindowArgs a) {
  constexpr int C = W + 1;
  __shared__ uint64_t s_bases[kBaseWords];
  __shared__ uint64_t s_hq[kPlaneWords];
  __shared__ uint64_t s_bad[kPlaneWords];
  __shared__ uint64_t s_st[kPlaneWords];
  __shared__ uint64_t s_red[kBlock / 64];
  __shared__ unsigned long long s_tag[kAggSlots];  // (tag << 32) | (position + 1), 0 = empty
  __shared__ uint32_t s_cnt[kAggSlots];
  __shared__ uint32_t s_tal[kAggSlots][4];  // left tally in the low, right in the high 16 bits
  PassCounts pc;
  const uint32_t k = a.k;
  const int ws = table_chunks(k);
  const SlotLayout lay = slot_layout(ws);
  const int64_t n_tiles = (a.n + kTile - 1) / kTile;
  const int64_t tpb = a.tiles_per_block > 0 ? a.tiles_per_block : 1;
  const int64_t t_end = min(n_tiles, ((int64_t)blockIdx.x + 1) * tpb);
  for (int64_t t = (int64_t)blockIdx.x * tpb; t < t_end; ++t) {
    const int64_t P0 = t * kTile, O = P0 - kHalo;
    __syncthreads();  // the previous tile's map is flushed
    stage_tile(a.bases, a.hq, a.bad, a.st, a.base_words, a.plane_words, O, s_bases, s_hq,
               s_bad, s_st);
    for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
      s_tag[i] = 0ull;
      s_cnt[i] = 0u;
#pragma unroll
      for (int b = 0; b < 4; ++b) s_tal[i][b] = 0u;
    }
    __syncthreads();
    for (int w0 = 0; w0 < kTile; w0 += kBlock) {
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      const int64_t p = P0 + w0 + tid;
      bool ok = false;
      uint64_t ch[C], hh = 0;
      bool use_rc = false;
      int L = -1, R = -1;
      const uint32_t lp = (uint32_t)(p - O);
      if (p + (int64_t)k <= a.n && !any_bits(s_bad, lp, k) && !any_bits(s_st, lp + 1, k - 1)) {
        staged_key<W, C>(s_bases, lp, k, ws, ch, hh, use_rc);
        ok = true;
        ++pc.win;
        int l = -1, rr = -1;
        if (!get_bit(s_st, lp) && get_bit(s_hq, lp - 1)) l = (int)get_base(s_bases, lp - 1);
        if (p + (int64_t)k < a.n && !get_bit(s_st, lp + k) && get_bit(s_hq, lp + k))
          rr = (int)get_base(s_bases, lp + k);
        L = use_rc ? (rr >= 0 ? 3 - rr : -1) : l;
        R = use_rc ? (l >= 0 ? 3 - l : -1) : rr;
      }
      // Bloom screen, as in the plain counting pass
      bool known = false;
      if (a.seen) {
        const uint64_t m = a.seen[(P0 + w0 + (tid & ~63)) >> 6];
        known = (m >> (tid & 63)) & 1;
      }
      if (ok && !known) {
        uint64_t blk;
        uint32_t pat;
        bloom_slot(hh, a.bloom_blocks, blk, pat);
        if (((uint32_t)(a.bloom[blk] >> 32) & pat) != pat) ok = false;
      }
      if (!ok) continue;
      ++pc.pass;
      // merge into the tile's map
      const uint32_t tag = (uint32_t)(hh >> 32) | 1u;
      const unsigned long long mine =
          ((unsigned long long)tag << 32) | (unsigned long long)(w0 + tid + 1);
      uint32_t x = (uint32_t)hh & (kAggSlots - 1);
      int slot = -1;
      for (int probe = 0; probe < kAggProbe; ++probe) {
        unsigned long long v = s_tag[x];
        if (v == 0ull) {
          v = atomicCAS(&s_tag[x], 0ull, mine);
          if (v == 0ull) {
            slot = (int)x;
            break;
          }
        }
        if ((uint32_t)(v >> 32) == tag) {  // same tag: compare with the claimer's key
          const uint32_t rp = (uint32_t)(v & 0xffffffffull) - 1u;
          uint64_t rch[C], rh;
          bool rrc;
          staged_key<W, C>(s_bases, (uint32_t)(P0 + rp - O), k, ws, rch, rh, rrc);
          bool eq = true;
#pragma unroll
          for (int c = 0; c < C; ++c) eq = eq && (c >= ws || rch[c] == ch[c]);
          if (eq) {
            slot = (int)x;
            break;
          }
        }
        x = (x + 1) & (kAggSlots - 1);
      }
      if (slot >= 0) {
        atomicAdd(&s_cnt[slot], 1u);
        if (L >= 0) atomicAdd(&s_tal[slot][L], 1u);
        if (R >= 0) atomicAdd(&s_tal[slot][R], 1u << 16);
        continue;
      }
      // no entry within the probe limit: update the table directly
      uint64_t w0w[C];
      const uint64_t s0 = __umul64hi(hh, a.capacity);
      load_slot_words<C>(a.table + s0 * lay.stride, ws, w0w);
      uint8_t* sp = find_or_claim<C>(a.table, a.capacity, lay.stride, ch, ws, s0, w0w,
                                     a.max_probe, pc.claim);
      if (!sp) {
        pc.fail = true;
        continue;
      }
      const uint32_t one_l[4] = {L == 0 ? 1u : 0u, L == 1 ? 1u : 0u, L == 2 ? 1u : 0u,
                                 L == 3 ? 1u : 0u};
      const uint32_t one_r[4] = {R == 0 ? 1u : 0u, R == 1 ? 1u : 0u, R == 2 ? 1u : 0u,
                                 R == 3 ? 1u : 0u};
      agg_update<C>(sp, lay, 1u, one_l, one_r);
    }
    __syncthreads();
    // flush: one table update per distinct k-mer of the tile
    for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
      const unsigned long long v = s_tag[i];
      if (v == 0ull) continue;
      const uint32_t rp = (uint32_t)(v & 0xffffffffull) - 1u;
      uint64_t ch[C], hh;
      bool rc_;
      staged_key<W, C>(s_bases, (uint32_t)(P0 + rp - O), k, ws, ch, hh, rc_);
      uint64_t w0w[C];
      const uint64_t s0 = __umul64hi(hh, a.capacity);
      load_slot_words<C>(a.table + s0 * lay.stride, ws, w0w);
      uint8_t* sp = find_or_claim<C>(a.table, a.capacity, lay.stride, ch, ws, s0, w0w,
                                     a.max_probe, pc.claim);
      if (!sp) {
        pc.fail = true;
        continue;
      }
      uint32_t l[4], r[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        l[b] = s_tal[i][b] & 0xffffu;
        r[b] = s_tal[i][b] >> 16;
      }
      agg_update<C>(sp, lay, s_cnt[i], l, r);
    }
  }
  flush_counts<2>(pc, a.ctr, nullptr, a.count_windows, s_red);
}

// A value known to be the same in every lane, moved to scalar registers.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

template <int W, int J>
__device__ __forceinline__ void bloom_slot_pass(const MultiBloomArgs& a, int ki,
                                                const uint64_t* s_bases,
                                                const uint64_t* s_hq,
                                                const uint64_t* s_bad,
                                                const uint64_t* s_st, int64_t P0,
                                                int64_t O, PassCounts& pc, int tid) {
  // the slot is the same for every lane: keep its fields in scalar registers
  const BloomSlot& sl = a.slots[ki];
  const uint32_t k = (uint32_t)__builtin_amdgcn_readfirstlane((int)sl.k);
  uint64_t* bloom = reinterpret_cast<uint64_t*>(uniform_u64((uint64_t)sl.bloom));
  const uint64_t blocks = uniform_u64(sl.bloom_blocks);
  uint64_t* seen = reinterpret_cast<uint64_t*>(uniform_u64((uint64_t)sl.seen));
  for (int w0 = 0; w0 < kTile; w0 += J * kBlock)
    tile_pass<W, 1, J>(s_bases, s_hq, s_bad, s_st, P0, O, w0, a.n, k, bloom, blocks, seen,
                       nullptr, 0, 0, nullptr, nullptr, 0, pc, nullptr, nullptr, 0, 0, tid,
                       a.shards, a.owner);
}

template <int W, int J>
__device__ __forceinline__ void bloom_slot_flush(const MultiBloomArgs& a, int ki,
                                                 const PassCounts& pc, uint64_t* s_red) {
  unsigned long long* ctr =
      reinterpret_cast<unsigned long long*>(uniform_u64((uint64_t)a.slots[ki].ctr));
  flush_counts<1>(pc, ctr, nullptr, 1, s_red);
  __syncthreads();  // s_red is reused by the next k
}

// Bloom pass A for up to kBloomFuse k of the same key width at once: each
// block stages a tile once and records the sightings of every k's windows
// in that k's filter; block b takes tiles b, b + grid, ...  (Mixing key
// widths in one kernel would make the compiler hold the registers of every
// width at once.)
template <int W, int J>
__global__ __launch_bounds__(kBlock) void k_bloom_multi(MultiBloomArgs a) {
  __shared__ uint64_t s_bases[kBaseWords];
  __shared__ uint64_t s_hq[kPlaneWords];
  __shared__ uint64_t s_bad[kPlaneWords];
  __shared__ uint64_t s_st[kPlaneWords];
  __shared__ uint64_t s_red[kBlock / 64];
  PassCounts pc0, pc1, pc2;
  const int64_t n_tiles = a.t_end > 0 ? a.t_end : (a.n + kTile - 1) / kTile;
  for (int64_t t = a.t_begin + blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t P0 = t * kTile, O = P0 - kHalo;
    __syncthreads();  // every window of the previous tile is formed
    stage_tile(a.bases, a.hq, a.bad, a.st, a.base_words, a.plane_words, O, s_bases, s_hq,
               s_bad, s_st);
    __syncthreads();
    // Straight-line calls (not a loop over k): each k's registers are dead
    // before the next k starts, so the kernel keeps the occupancy of a
    // single-k pass.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    bloom_slot_pass<W, J>(a, 0, s_bases, s_hq, s_bad, s_st, P0, O, pc0, tid);
    if (a.nk > 1) bloom_slot_pass<W, J>(a, 1, s_bases, s_hq, s_bad, s_st, P0, O, pc1, tid);
    if (a.nk > 2) bloom_slot_pass<W, J>(a, 2, s_bases, s_hq, s_bad, s_st, P0, O, pc2, tid);
  }
  bloom_slot_flush<W, J>(a, 0, pc0, s_red);
  if (a.nk > 1) bloom_slot_flush<W, J>(a, 1, pc1, s_red);
  if (a.nk > 2) bloom_slot_flush<W, J>(a, 2, pc2, s_red);
}

// Grid of a launch over `n_tiles` tiles taking `tiles_per_block` each.
// Blocks of a grid-stride window pass: tiles_per_block tiles each, but at
// least four blocks per compute unit while there are that many tiles (a
// tuning chosen for a large read set would otherwise leave most of the
// chip idle on a small one).
static unsigned grid_of(int64_t n_tiles, int tiles_per_block) {
  constexpr int64_t kMinBlocks = 1024;
  int64_t t = tiles_per_block > 0 ? tiles_per_block : 1;
  t = std::min<int64_t>(t, std::max<int64_t>(1, n_tiles / kMinBlocks));
  return (unsigned)((n_tiles + t - 1) / t);
}

template <int W>
static void launch_bloom_multi_w(const MultiBloomArgs& a, unsigned blocks, hipStream_t s) {
  if (a.lanes == 1)
    hipLaunchKernelGGL((k_bloom_multi<W, 1>), dim3(blocks), dim3(kBlock), 0, s, a);
  else if (a.lanes == 2)
    hipLaunchKernelGGL((k_bloom_multi<W, 2>), dim3(blocks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_bloom_multi<W, 4>), dim3(blocks), dim3(kBlock), 0, s, a);
}

void launch_bloom_multi(const MultiBloomArgs& a, hipStream_t s) {
  // all k of the launch have the key width of a.k0
  const int64_t t_end = a.t_end > 0 ? a.t_end : (a.n + kTile - 1) / kTile;
  if (t_end <= a.t_begin) return;
  const unsigned blocks = grid_of(t_end - a.t_begin, a.tiles_per_block);
  if (blocks == 0 || a.nk == 0) return;
  switch ((a.k0 + 31) / 32) {
    case 1: launch_bloom_multi_w<1>(a, blocks, s); break;
    case 2: launch_bloom_multi_w<2>(a, blocks, s); break;
    case 3: launch_bloom_multi_w<3>(a, blocks, s); break;
    default: launch_bloom_multi_w<4>(a, blocks, s); break;
  }
}

// Windows per lane when the tuning leaves it to the key width (lanes 0):
// two for two- and three-word keys, whose counting passes were measured
// ~25-35 % faster so on the 10M-read metagenome, one otherwise.
template <int W>
constexpr int lanes_for_width() {
  return (W == 2 || W == 3) ? 2 : 1;
}

template <int W, int MODE>
static void launch_windows_wm(const WindowArgs& a, unsigned blocks, hipStream_t s) {
  const int lanes = a.lanes ? a.lanes : lanes_for_width<W>();
  if (lanes == 1)
    hipLaunchKernelGGL((k_windows<W, MODE, 1>), dim3(blocks), dim3(kBlock), 0, s, a);
  else if (lanes == 2)
    hipLaunchKernelGGL((k_windows<W, MODE, 2>), dim3(blocks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_windows<W, MODE, 4>), dim3(blocks), dim3(kBlock), 0, s, a);
}

template <int W>
static void launch_windows_w(const WindowArgs& a, int mode, hipStream_t s) {
  const int64_t t_end = a.t_end > 0 ? a.t_end : (a.n + kTile - 1) / kTile;
  if (!a.tiles && t_end <= a.t_begin) return;
  const unsigned blocks = a.tiles ? (unsigned)a.n_tiles
                                  : grid_of(t_end - a.t_begin, a.tiles_per_block);
  if (blocks == 0) return;
  if (mode == 0)
    launch_windows_wm<W, 0>(a, blocks, s);
  else if (mode == 1)
    launch_windows_wm<W, 1>(a, blocks, s);
  else if (mode == 2 && a.aggregate && !a.tiles && a.shards <= 1 && W <= 3)
    hipLaunchKernelGGL((k_count_agg<W>), dim3(blocks), dim3(kBlock), 0, s, a);
  else if (mode == 2)
    launch_windows_wm<W, 2>(a, blocks, s);
  else
    launch_windows_wm<W, 3>(a, blocks, s);
}

void launch_windows(const WindowArgs& a, int mode, hipStream_t s) {
  switch ((a.k + 31) / 32) {
    case 1: launch_windows_w<1>(a, mode, s); break;
    case 2: launch_windows_w<2>(a, mode, s); break;
    case 3: launch_windows_w<3>(a, mode, s); break;
    default: launch_windows_w<4>(a, mode, s); break;
  }
}

// ------------------------------------------------------------- replay ----

// One thread per overflow entry: re-form the window straight from the
// descriptor's planes in HBM (the same bit arithmetic as the staged tile, at
// the global position) and count it into the grown table.
template <int W>
__global__ __launch_bounds__(kBlock) void k_replay(const TileDesc* __restrict__ descs,
                                                   const uint64_t* __restrict__ entries,
                                                   uint64_t n, uint32_t k) {
  constexpr int C = W + 1;
  const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const uint64_t v = entries[e];
  const TileDesc& d = descs[v >> 10];
  const int64_t p = d.p0 + (int64_t)(v & 1023);
  const int ws = table_chunks(k);
  const SlotLayout lay = slot_layout(ws);
  // the entry was a valid window when it was recorded
  uint64_t f[W], r[W], key[W];
  // positions are global here: start the extraction at the window's word
  window_words<W>(d.bases + ((2 * p) >> 6), (uint32_t)((2 * p) & 63), k, f);
  revcomp_words<W>(f, k, r);
  const bool use_rc = words_less<W>(r, f);
#pragma unroll
  for (int w = 0; w < W; ++w) key[w] = use_rc ? r[w] : f[w];
  uint64_t ch[C];
  to_chunks<W, C>(key, ws, ch);
  const uint64_t h = hash_chunks<C>(ch, ws);
  int l = -1, rr = -1;
  {
    const bool start = (d.st[p >> 6] >> (63 - (p & 63))) & 1;
    if (!start && p >= 1) {
      const int64_t q = p - 1;
      if ((d.hq[q >> 6] >> (63 - (q & 63))) & 1)
        l = (int)((d.bases[q >> 5] >> (62 - 2 * (q & 31))) & 3);
    }
    const int64_t q = p + (int64_t)k;
    if (q < d.hi) {
      const bool qs = (d.st[q >> 6] >> (63 - (q & 63))) & 1;
      const bool qh = (d.hq[q >> 6] >> (63 - (q & 63))) & 1;
      if (!qs && qh) rr = (int)((d.bases[q >> 5] >> (62 - 2 * (q & 31))) & 3);
    }
  }
  int L = l, R = rr;
  if (use_rc) {
    L = rr >= 0 ? 3 - rr : -1;
    R = l >= 0 ? 3 - l : -1;
  }
  uint32_t claimed = 0;
  const uint64_t i0 = __umul64hi(h, d.capacity);
  uint64_t w0[C];
  load_slot_words<C>(d.table + i0 * lay.stride, ws, w0);
  uint8_t* sp = find_or_claim<C>(d.table, d.capacity, lay.stride, ch, ws, i0, w0,
                                 d.capacity < 0xffffffffull ? (uint32_t)d.capacity : 0xffffffffu,
                                 claimed);
  if (!sp) return;  // cannot happen: the table has a free slot for every entry
  if (claimed) atomicAdd(&d.counters[0], (unsigned long long)claimed);
  const uint64_t old = __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(sp + lay.x_off),
                                              x_increment(L, R), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t c = (uint32_t)(old & kCountMask);
  if (c >= kSpillAt) {
    if (L >= 0)
      __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(sp + lay.sl_off), 1ull << (16 * L),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (R >= 0)
      __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(sp + lay.sr_off), 1ull << (16 * R),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (c == kHeavyCount - 1)
      __hip_atomic_fetch_or(reinterpret_cast<uint64_t*>(sp + lay.sr_off), kHeavyBit,
                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

void launch_replay(const TileDesc* descs, const uint64_t* entries, uint64_t n,
                   uint32_t k, hipStream_t s) {
  if (n == 0) return;
  const dim3 g((unsigned)((n + kBlock - 1) / kBlock));
  switch ((k + 31) / 32) {
    case 1: hipLaunchKernelGGL(k_replay<1>, g, dim3(kBlock), 0, s, descs, entries, n, k); break;
    case 2: hipLaunchKernelGGL(k_replay<2>, g, dim3(kBlock), 0, s, descs, entries, n, k); break;
    case 3: hipLaunchKernelGGL(k_replay<3>, g, dim3(kBlock), 0, s, descs, entries, n, k); break;
    default: hipLaunchKernelGGL(k_replay<4>, g, dim3(kBlock), 0, s, descs, entries, n, k); break;
  }
}

// ------------------------------------------------------------- rehash ----

// One thread per old slot: claim the key's slot in the new table (keys are
// unique, so every claim succeeds on an empty or fresh slot) and copy the
// packed counter and spill words.
template <int C>
__global__ __launch_bounds__(kBlock) void k_rehash(const uint8_t* __restrict__ old_t,
                                                   uint64_t old_cap,
                                                   uint8_t* __restrict__ new_t,
                                                   uint64_t new_cap, uint32_t k,
                                                   unsigned long long* ctr) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= old_cap) return;
  const int ws = table_chunks(k);
  const SlotLayout lay = slot_layout(ws);
  const uint8_t* os = old_t + i * lay.stride;
  const uint64_t* oc = reinterpret_cast<const uint64_t*>(os);
  if (oc[0] == 0) return;
  uint64_t ch[C];
#pragma unroll
  for (int c = 0; c < C; ++c) ch[c] = c < ws ? oc[c] : 0ull;
  const uint64_t h = hash_chunks<C>(ch, ws);
  const uint64_t s0 = __umul64hi(h, new_cap);
  uint32_t claimed = 0;
  uint64_t w0[C];
  load_slot_words<C>(new_t + s0 * lay.stride, ws, w0);
  uint8_t* ns = find_or_claim<C>(new_t, new_cap, lay.stride, ch, ws, s0, w0,
                                 new_cap < 0xffffffffull ? (uint32_t)new_cap : 0xffffffffu,
                                 claimed);
  if (!ns) {
    atomicOr(&ctr[kCtrStatus], (unsigned long long)kStatusProbeLimit);
    return;
  }
  *reinterpret_cast<uint64_t*>(ns + lay.x_off) = *reinterpret_cast<const uint64_t*>(os + lay.x_off);
  *reinterpret_cast<uint64_t*>(ns + lay.sl_off) = *reinterpret_cast<const uint64_t*>(os + lay.sl_off);
  *reinterpret_cast<uint64_t*>(ns + lay.sr_off) = *reinterpret_cast<const uint64_t*>(os + lay.sr_off);
}

void launch_rehash(const uint8_t* old_table, uint64_t old_cap, uint8_t* new_table,
                   uint64_t new_cap, uint32_t k, unsigned long long* ctr,
                   hipStream_t s) {
  if (old_cap == 0) return;
  const dim3 g((unsigned)((old_cap + kBlock - 1) / kBlock));
  switch ((k + 31) / 32) {
    case 1: hipLaunchKernelGGL(k_rehash<2>, g, dim3(kBlock), 0, s, old_table, old_cap, new_table, new_cap, k, ctr); break;
    case 2: hipLaunchKernelGGL(k_rehash<3>, g, dim3(kBlock), 0, s, old_table, old_cap, new_table, new_cap, k, ctr); break;
    case 3: hipLaunchKernelGGL(k_rehash<4>, g, dim3(kBlock), 0, s, old_table, old_cap, new_table, new_cap, k, ctr); break;
    default: hipLaunchKernelGGL(k_rehash<5>, g, dim3(kBlock), 0, s, old_table, old_cap, new_table, new_cap, k, ctr); break;
  }
}

// ----------------------------------------------------- classify/compact ----

// Top min(64, 2k) bits of a key given as W export words (the sort key).
template <int W>
__device__ __forceinline__ uint64_t key_prefix(const uint64_t (&f)[W], uint32_t k) {
  if (W == 1) return f[0];
  const uint32_t bits0 = 2u * k - 64u * (W - 1);  // 2..62 for odd k
  return (f[0] << (64 - bits0)) | (f[1] >> bits0);
}

// Keep occupied slots with count >= min_count: write their key prefix (the
// sort key) and their slot index.  Each block takes chunks of kClassifyItems
// slots per thread; output positions come from a block-wide prefix sum and
// one atomic per chunk (row order is arbitrary here; the sort fixes it).
constexpr int kClassifyItems = 8;

template <int W>
__global__ __launch_bounds__(kBlock) void k_classify(ClassifyArgs a) {
  __shared__ uint32_t s_wave[kBlock / 64];
  __shared__ uint64_t s_base;
  const int ws = table_chunks(a.k);
  const SlotLayout lay = slot_layout(ws);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t chunk = (uint64_t)kBlock * kClassifyItems;
  for (uint64_t c0 = (uint64_t)blockIdx.x * chunk; c0 < a.capacity;
       c0 += (uint64_t)gridDim.x * chunk) {
    // Each kept slot's sort key is formed right after its test, while the
    // slot's line is still cached (forming it after the block's prefix sum
    // fetched many lines a second time).
    uint32_t keep = 0, heavy = 0, n = 0;
    uint64_t pfx[kClassifyItems];
#pragma unroll
    for (int it = 0; it < kClassifyItems; ++it) {
      pfx[it] = 0;
      const uint64_t i = c0 + (uint64_t)it * kBlock + tid;
      if (i < a.capacity) {
        const uint8_t* s = a.table + i * lay.stride;
        const uint64_t w0 = *reinterpret_cast<const uint64_t*>(s);
        const uint64_t xw = *reinterpret_cast<const uint64_t*>(s + lay.x_off);
        const uint64_t sr = *reinterpret_cast<const uint64_t*>(s + lay.sr_off);
        // a heavy k-mer has count >= kHeavyCount >= min_count
        if (w0 != 0 && ((sr & kHeavyBit) || (uint32_t)(xw & kCountMask) >= a.min_count)) {
          keep |= 1u << it;
          if (sr & kHeavyBit) heavy |= 1u << it;
          ++n;
          uint64_t f[W];
          from_chunks<W>(reinterpret_cast<const uint64_t*>(s), ws, f);
          pfx[it] = W == 1 ? f[0] : key_prefix<W>(f, a.k) >> (64 - kSortPrefixBits);
        }
      }
    }
    // block-exclusive prefix of n
    uint32_t incl = n;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t off = incl - n, total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      if (w < wave) off += s_wave[w];
      total += s_wave[w];
    }
    if (tid == 0) s_base = total ? atomicAdd(&a.ctr[kCtrRows], (unsigned long long)total) : 0ull;
    __syncthreads();
    uint64_t pos = s_base + off;
#pragma unroll
    for (int it = 0; it < kClassifyItems; ++it) {
      if (keep & (1u << it)) {
        const uint64_t i = c0 + (uint64_t)it * kBlock + tid;
        if (heavy & (1u << it)) {  // fields may have wrapped: recount exactly later
          atomicOr(&a.ctr[kCtrStatus], (unsigned long long)kStatusHeavy);
          const uint64_t hp = atomicAdd(&a.ctr[kCtrHeavy], 1ull);
          if (hp < kHeavyMax) a.heavy_list[hp] = (uint32_t)i;
        }
        a.pfx_out[pos] = pfx[it];
        a.idx_out[pos] = (uint32_t)i;
        ++pos;
      }
    }
    __syncthreads();  // s_wave / s_base are rewritten by the next chunk
  }
}

void launch_classify(const ClassifyArgs& a, hipStream_t s) {
  if (a.capacity == 0) return;
  const uint64_t chunk = (uint64_t)kBlock * kClassifyItems;
  uint64_t blocks = (a.capacity + chunk - 1) / chunk;
  if (blocks > 8192) blocks = 8192;
  switch ((a.k + 31) / 32) {
    case 1: hipLaunchKernelGGL(k_classify<1>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_classify<2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_classify<3>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
    default: hipLaunchKernelGGL(k_classify<4>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
  }
}

// ------------------------------------------------------------ tie runs ----

template <int W>
__device__ __forceinline__ void slot_key(const uint8_t* table, uint32_t stride,
                                         int ws, uint32_t slot, uint64_t (&f)[W]) {
  from_chunks<W>(reinterpret_cast<const uint64_t*>(table + (uint64_t)slot * stride),
                 ws, f);
}

// One thread per row: the first row of a run of equal prefixes insertion-sorts
// the run's slot indices by full key (runs are short: equal top 20 bases).
template <int W>
__global__ __launch_bounds__(kBlock) void k_fix_ties(
    const uint64_t* __restrict__ pfx, uint32_t* __restrict__ idx, int64_t n,
    const uint8_t* __restrict__ table, uint32_t k,
    unsigned long long* __restrict__ ctr) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i + 1 >= n) return;
  const uint64_t p = pfx[i];
  if (pfx[i + 1] != p || (i > 0 && pfx[i - 1] == p)) return;
  int64_t j = i + 2;
  while (j < n && j - i <= kMaxTieRun && pfx[j] == p) ++j;
  if (j - i > kMaxTieRun) {
    atomicOr(&ctr[kCtrStatus], (unsigned long long)kStatusLongTies);
    return;
  }
  const int ws = table_chunks(k);
  const uint32_t stride = slot_layout(ws).stride;
  for (int64_t a = i + 1; a < j; ++a) {
    const uint32_t cur = idx[a];
    uint64_t fc[W];
    slot_key<W>(table, stride, ws, cur, fc);
    int64_t b = a - 1;
    while (b >= i) {
      uint64_t fb[W];
      slot_key<W>(table, stride, ws, idx[b], fb);
      if (!words_less<W>(fc, fb)) break;
      idx[b + 1] = idx[b];
      --b;
    }
    idx[b + 1] = cur;
  }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_row_keys(
    const uint32_t* __restrict__ idx, int64_t n, const uint8_t* __restrict__ table,
    uint32_t k, uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int ws = table_chunks(k);
  uint64_t f[W];
  slot_key<W>(table, slot_layout(ws).stride, ws, idx[i], f);
#pragma unroll
  for (int w = 0; w < W; ++w) keys[i * W + w] = f[w];
}

void launch_fix_ties(const uint64_t* pfx, uint32_t* idx, int64_t n,
                     const uint8_t* table, uint32_t k, unsigned long long* ctr,
                     hipStream_t s) {
  if (n < 2 || 2 * k <= 64) return;  // sort keys are whole keys: no ties
  const dim3 g((unsigned)((n + kBlock - 1) / kBlock));
  switch ((k + 31) / 32) {
    case 2: hipLaunchKernelGGL(k_fix_ties<2>, g, dim3(kBlock), 0, s, pfx, idx, n, table, k, ctr); break;
    case 3: hipLaunchKernelGGL(k_fix_ties<3>, g, dim3(kBlock), 0, s, pfx, idx, n, table, k, ctr); break;
    default: hipLaunchKernelGGL(k_fix_ties<4>, g, dim3(kBlock), 0, s, pfx, idx, n, table, k, ctr); break;
  }
}

void launch_row_keys(const uint32_t* idx, int64_t n, const uint8_t* table,
                     uint32_t k, uint64_t* keys, hipStream_t s) {
  if (n == 0) return;
  const dim3 g((unsigned)((n + kBlock - 1) / kBlock));
  switch ((k + 31) / 32) {
    case 1: hipLaunchKernelGGL(k_row_keys<1>, g, dim3(kBlock), 0, s, idx, n, table, k, keys); break;
    case 2: hipLaunchKernelGGL(k_row_keys<2>, g, dim3(kBlock), 0, s, idx, n, table, k, keys); break;
    case 3: hipLaunchKernelGGL(k_row_keys<3>, g, dim3(kBlock), 0, s, idx, n, table, k, keys); break;
    default: hipLaunchKernelGGL(k_row_keys<4>, g, dim3(kBlock), 0, s, idx, n, table, k, keys); break;
  }
}

// --------------------------------------------------------- heavy build ----

// One thread per heavy k-mer: copy its stored key into a heavy entry, index
// the entry by hash, and leave the entry number in the slot's SL word (the
// packed tallies of a heavy slot are no longer used).
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
  e.count = 0;
  for (int j = 0; j < 8; ++j) e.ext[j] = 0;
  uint64_t hh = 0x9e3779b97f4a7c15ull;
  for (int j = 0; j < ws; ++j) hh = fmix64(hh ^ c[j]);
  uint32_t x = (uint32_t)(hh >> 32) & a.heavy_mask;
  for (uint32_t probe = 0; probe <= a.heavy_mask; ++probe) {
    if (atomicCAS(&a.heavy_index[x], kHeavyEmpty, h) == kHeavyEmpty) break;
    x = (x + 1) & a.heavy_mask;
  }
  *reinterpret_cast<uint64_t*>(s + lay.sl_off) = (uint64_t)h;
}

void launch_heavy_build(const HeavyBuildArgs& a, hipStream_t s) {
  if (a.n_heavy == 0) return;
  hipLaunchKernelGGL(k_heavy_build, dim3((a.n_heavy + kBlock - 1) / kBlock),
                     dim3(kBlock), 0, s, a);
}

// ------------------------------------------------------------- gather ----

template <int W>
__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs a) {
  // One row per thread.  Its slot is read whole with 16-byte loads: one-word
  // keys (odd k <= 31) have one stored chunk and 32-byte slots (chunk, X,
  // SL, SR), wider keys 64-byte slots (chunks, then X, SL, SR in the last
  // three words), as slot_layout gives them.
  constexpr int NW = W == 1 ? 4 : 8;
  const int ws = table_chunks(a.k);
  const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (row >= a.n_rows) return;
  const uint4* sv = reinterpret_cast<const uint4*>(a.table + (uint64_t)a.idx[row] * (NW * 8));
  uint64_t sw[NW];
#pragma unroll
  for (int i = 0; i < NW / 2; ++i) {
    const uint4 v = sv[i];
    sw[2 * i] = (uint64_t)v.x | ((uint64_t)v.y << 32);
    sw[2 * i + 1] = (uint64_t)v.z | ((uint64_t)v.w << 32);
  }
  {  // the key from its 62-bit chunks, least significant chunk first
    uint64_t lw[W];
#pragma unroll
    for (int j = 0; j < W; ++j) lw[j] = 0;
#pragma unroll
    for (int cc = 0; cc < W + 1; ++cc) {
      if (cc < ws) {
        const uint64_t v = sw[cc] & kMask62;
        const int lo = 62 * cc, wi = lo >> 6, off = lo & 63;
#pragma unroll
        for (int j = 0; j < W; ++j) {
          if (j == wi) lw[j] |= v << off;
          if (j == wi + 1 && off > 2) lw[j] |= v >> (64 - off);
        }
      }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) a.keys[row * W + w] = lw[W - 1 - w];
  }
  const uint64_t xw = sw[NW - 3], sl = sw[NW - 2], sr = sw[NW - 1];
  uint32_t l[4], r[4], cnt;
  if (sr & kHeavyBit) {  // heavy hitter: exact count and tallies from the recount
    const HeavyEntry& e = a.heavy[sl];
    cnt = e.count;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      l[b] = e.ext[b];
      r[b] = e.ext[4 + b];
    }
  } else {
    decode_slot(xw, sl, sr, cnt, l, r);
  }
  a.counts[row] = cnt;
  uint4* e = reinterpret_cast<uint4*>(a.ext + row * 8);
  e[0] = make_uint4(l[0], l[1], l[2], l[3]);
  e[1] = make_uint4(r[0], r[1], r[2], r[3]);
  // both letters in one 2-byte store (left letter first in memory)
  reinterpret_cast<uint16_t*>(a.codes)[row] =
      (uint16_t)((uint32_t)side_code(l, cnt, a.t_min_ext, a.t_base, a.err_ppm) |
                 ((uint32_t)side_code(r, cnt, a.t_min_ext, a.t_base, a.err_ppm) << 8));
}

void launch_gather(const GatherArgs& a, hipStream_t s) {
  if (a.n_rows == 0) return;
  const dim3 g((unsigned)((a.n_rows + kBlock - 1) / kBlock));
  switch ((a.k + 31) / 32) {
    case 1: hipLaunchKernelGGL(k_gather<1>, g, dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_gather<2>, g, dim3(kBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_gather<3>, g, dim3(kBlock), 0, s, a); break;
    default: hipLaunchKernelGGL(k_gather<4>, g, dim3(kBlock), 0, s, a); break;
  }
}

}  // namespace kh
