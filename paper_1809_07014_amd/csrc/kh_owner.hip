// Owner-partitioned counting: the k-mer analysis of Section II-B laid out the
// way the paper distributes it.  There, every k-mer is sent to the process
// that owns it, and each owner runs the two-pass Bloom screen and the
// hash-table count over its own k-mers in local memory.  Here an owner is a
// range of key prefixes small enough for one workgroup, and the owner's local
// memory is that workgroup's LDS.
//
// Routing (the all-to-all exchange of the paper) is two streaming radix
// partitions over the key prefix: the windows' records go to 2^p1 level-1
// buckets (the top p1 key bits), then each bucket is split by its next p2_b
// bits into owners of a few thousand records (p2_b chosen per bucket from its
// size).  Every pass writes contiguous runs at offsets from a scanned
// histogram matrix, so no device-scope atomic touches a random address.  An
// owner workgroup then runs Bloom pass A and count pass B over its records in
// LDS and classifies the kept k-mers; the copy of the owners' rows into the
// table sorts each owner's rows, and the owners' prefixes are disjoint and in
// key order, so sorting within owners orders the whole table.
//
// A record is one window: its canonical key without the level-1 digit (the
// bucket implies those bits), shifted left by 6 bits with the extension byte
// (left valid, left base, right valid, right base) below it, as
// R = own_record_words(k) words, most significant first.  Owners count these
// partial keys (they share the digit) and put the digit back when
// they write their rows.
#include "kh_internal.hpp"

namespace kh {

// ------------------------------------------------------------ helpers ----

// Bits [pos, pos + len) (MSB-first, 0 <= len <= 32) of an N-word value held
// in registers, most significant word first.  Indexes are static.
template <int N>
__device__ __forceinline__ uint32_t top_bits(const uint64_t (&v)[N], int pos, int len) {
  if (len <= 0) return 0u;
  const int q = pos >> 6, r = pos & 63;
  uint64_t hi = 0;
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i == q) hi = v[i] << r;
  if (r + len > 64) {
#pragma unroll
    for (int i = 0; i + 1 < N; ++i)
      if (i == q) hi |= v[i + 1] >> (64 - r);
  }
  return (uint32_t)(hi >> (64 - len));
}

// (key << 6) | e6 as R words (R = W or W + 1).
template <int W, int R>
__device__ __forceinline__ void make_record(const uint64_t (&f)[W], uint32_t e6,
                                            uint64_t (&v)[R]) {
#pragma unroll
  for (int j = 0; j < R; ++j) {  // j counts words from the least significant
    const uint64_t cur = j < W ? f[W - 1 - j] : 0ull;
    const uint64_t low = j == 0 ? (uint64_t)e6 : (j - 1 < W ? f[W - j] >> 58 : 0ull);
    v[R - 1 - j] = (cur << 6) | low;
  }
}

// The key of a record (record >> 6) as R words, most significant first.
template <int R>
__device__ __forceinline__ void record_key(const uint64_t (&v)[R], uint64_t (&key)[R]) {
#pragma unroll
  for (int j = 0; j < R; ++j)
    key[j] = (v[j] >> 6) | (j > 0 ? v[j - 1] << 58 : 0ull);
}

template <int R>
__device__ __forceinline__ void load_record(const uint64_t* __restrict__ rec, uint64_t r,
                                            uint64_t (&v)[R]) {
  if (R == 2) {
    const uint4 x = reinterpret_cast<const uint4*>(rec)[r];
    v[0] = (uint64_t)x.x | ((uint64_t)x.y << 32);
    v[R - 1] = (uint64_t)x.z | ((uint64_t)x.w << 32);
  } else {
#pragma unroll
    for (int w = 0; w < R; ++w) v[w] = rec[r * R + w];
  }
}

// The canonical key and extension byte of the window at p (staged tile at
// O) whose forward words f and reverse complement r are known; false if it
// is not a k-mer or belongs to another key part.
template <int W>
__device__ __forceinline__ bool own_window_fr(const uint64_t* s_bases, const uint64_t* s_hq,
                                              const uint64_t* s_bad, const uint64_t* s_st,
                                              int64_t p, int64_t O, int64_t n_end, uint32_t k,
                                              uint32_t shards, uint32_t owner,
                                              const uint64_t (&f)[W], const uint64_t (&r)[W],
                                              uint64_t (&key)[W], uint32_t& e6,
                                              int lbase = -1, int rbase = -1) {
  if (p + (int64_t)k > n_end) return false;
  const uint32_t lp = (uint32_t)(p - O);
  if (any_bits(s_bad, lp, k) || any_bits(s_st, lp + 1, k - 1)) return false;
  const bool use_rc = words_less<W>(r, f);
#pragma unroll
  for (int w = 0; w < W; ++w) key[w] = use_rc ? r[w] : f[w];
  if (shards > 1 && owner_of<W>(key, shards) != owner) return false;
  // the neighbouring bases (the caller's, when it has them: lbase, rbase)
  int l = -1, rr = -1;
  if (!get_bit(s_st, lp) && get_bit(s_hq, lp - 1))
    l = lbase >= 0 ? lbase : (int)get_base(s_bases, lp - 1);
  if (p + (int64_t)k < n_end && !get_bit(s_st, lp + k) && get_bit(s_hq, lp + k))
    rr = rbase >= 0 ? rbase : (int)get_base(s_bases, lp + k);
  int L = l, Rt = rr;
  if (use_rc) {
    L = rr >= 0 ? 3 - rr : -1;
    Rt = l >= 0 ? 3 - l : -1;
  }
  e6 = (L >= 0 ? 32u | ((uint32_t)L << 3) : 0u) | (Rt >= 0 ? 4u | (uint32_t)Rt : 0u);
  return true;
}

// A window of the staged tile as its canonical key and extension byte
// (Section II-B: every k-mer of a read, its neighbours as extensions when
// they pass the quality cutoff; on the reverse strand the sides swap and
// complement).  False if it is not a k-mer or belongs to another key part.
template <int W>
__device__ __forceinline__ bool own_window(const uint64_t* s_bases, const uint64_t* s_hq,
                                           const uint64_t* s_bad, const uint64_t* s_st,
                                           int64_t p, int64_t O, int64_t n_end, uint32_t k,
                                           uint32_t shards, uint32_t owner,
                                           uint64_t (&key)[W], uint32_t& e6) {
  if (p + (int64_t)k > n_end) return false;
  const uint32_t lp = (uint32_t)(p - O);
  if (any_bits(s_bad, lp, k) || any_bits(s_st, lp + 1, k - 1)) return false;
  uint64_t f[W], r[W];
  window_words<W>(s_bases, 2 * lp, k, f);
  revcomp_words<W>(f, k, r);
  return own_window_fr<W>(s_bases, s_hq, s_bad, s_st, p, O, n_end, k, shards, owner, f, r, key,
                          e6);
}

// The next window's words: base b enters at the right of the forward words
// and, complemented, at the left of the reverse complement (k-base values,
// W words most significant first, the top word holding 2k - 64 (W - 1) bits).
template <int W>
__device__ __forceinline__ void roll_words(uint64_t (&f)[W], uint64_t (&r)[W], uint32_t b,
                                           uint32_t k) {
  const int tb = 2 * (int)k - 64 * (W - 1);  // 2 .. 64
  const uint64_t tmask = tb >= 64 ? ~0ull : (1ull << tb) - 1ull;
#pragma unroll
  for (int j = 0; j < W; ++j) f[j] = (f[j] << 2) | (j + 1 < W ? f[j + 1] >> 62 : (uint64_t)b);
  f[0] &= tmask;
#pragma unroll
  for (int j = W - 1; j > 0; --j) r[j] = (r[j] >> 2) | (r[j - 1] << 62);
  r[0] = (r[0] >> 2) | ((uint64_t)(3u - b) << (tb - 2));
}

// Level-1 bucket of the window at p without forming its key: the top p1
// bits of the canonical key are the smaller of the window's first p1 / 2
// bases and the reverse complement of its last p1 / 2 bases (when the two
// are equal, the key starts with them whichever strand it is read on).
// -1 if the window is not a k-mer.
__device__ __forceinline__ int own_top(const uint64_t* s_bases, const uint64_t* s_bad,
                                       const uint64_t* s_st, int64_t p, int64_t O,
                                       int64_t n_end, uint32_t k, int p1) {
  if (p + (int64_t)k > n_end) return -1;
  const uint32_t lp = (uint32_t)(p - O);
  if (any_bits(s_bad, lp, k) || any_bits(s_st, lp + 1, k - 1)) return -1;
  const uint32_t nb = (uint32_t)p1 >> 1;
  const uint32_t f = (uint32_t)get_bits(s_bases, 2 * lp, (uint32_t)p1);
  const uint32_t t = (uint32_t)get_bits(s_bases, 2 * (lp + k - nb), (uint32_t)p1);
  // reverse the order of t's bases: reverse its bits, then swap each pair back
  uint32_t r = __builtin_bitreverse32(t) >> (32 - p1);
  r = ((r >> 1) & 0x55555555u) | ((r & 0x55555555u) << 1);
  r = ~r & ((1u << p1) - 1u);  // complement
  return (int)(f < r ? f : r);
}

// Records of a batch starting at record b0 that lane `tid` holds (records
// b0 + q x kOwnThreads + tid for q < the result, at most NB) when the
// owner's records end at r1.
template <int NB>
__device__ __forceinline__ int lane_records(uint64_t b0, uint64_t r1, int tid) {
  const uint64_t first = b0 + (uint64_t)tid;
  if (first >= r1) return 0;
  const uint64_t n = (r1 - first + kOwnThreads - 1) / kOwnThreads;
  return n < (uint64_t)NB ? (int)n : NB;
}

// Hash of a key held as stored chunks, for the LDS table and the Bloom
// filter of one owner (whose keys share their prefix; only the other bits
// vary): a multiply-add over the chunks and one xor-shift.  Slot index: its
// top 32 bits scaled to the table; Bloom word and four pattern bits: two
// 32-bit multiply-xorshift steps on its low half.
template <int C>
__device__ __forceinline__ uint64_t owner_hash(const uint64_t (&ch)[C], int ws) {
  const uint64_t K[5] = {0x9e3779b97f4a7c15ull, 0xc2b2ae3d27d4eb4full, 0x165667b19e3779f9ull,
                         0xd6e8feb86659fd93ull, 0xff51afd7ed558ccdull};
  uint64_t h = 0;
#pragma unroll
  for (int c = 0; c < C; ++c)
    if (c < ws) h += ch[c] * K[c];
  return h ^ (h >> 29);
}

__device__ __forceinline__ void owner_bloom(uint64_t h, uint32_t& bi, uint32_t& pat) {
  uint32_t t = (uint32_t)h * 0x85ebca6bu;
  t ^= t >> 13;
  bi = t >> (32 - kOwnBloomBits);
  const uint32_t u = (t ^ (t >> 16)) * 0xc2b2ae35u;
  pat = (1u << (u & 31)) | (1u << ((u >> 5) & 31)) | (1u << ((u >> 10) & 31)) |
        (1u << ((u >> 15) & 31));
}

// Barrier for LDS exchange only: it waits for this wave's LDS operations but
// not for its outstanding global loads and stores, which the fence in
// __syncthreads would wait for (a full memory round trip at every barrier).
// Used where the waves of a block share data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Exclusive scan of one value per thread over the block (blockDim.x a
// multiple of 64, at most 1024); returns the block total.  s_w holds one
// word per wave.  Every thread calls it.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& excl,
                                                    uint32_t* s_w) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x >> 6);
  uint32_t incl = x;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  lds_barrier();
  if (lane == 63) s_w[wave] = incl;
  lds_barrier();
  uint32_t off = 0, total = 0;
  for (int w = 0; w < nw; ++w) {
    const uint32_t s = s_w[w];
    if (w < wave) off += s;
    total += s;
  }
  excl = off + incl - x;
  return total;
}

// ------------------------------------------------------ level 1 route ----

// Routing tiles: kOwnTiles tiles of window starts staged at once, one
// window of each tile per lane.
constexpr int kOwnTiles = kOwnRouteThreads * 4 / kTile;
constexpr int kOwnSpan = kOwnTiles * kTile + 256;  // staged positions (k <= 127)
constexpr int kOwnBaseWords = kOwnSpan / 32 + 1;
constexpr int kOwnPlaneWords = kOwnSpan / 64 + 1;
constexpr int kOwnTile = kOwnTiles * kTile;        // window starts per routing tile

// Stage the planes of positions [O, O + kOwnSpan) (as stage_tile: outside the
// read set no bases, every position bad).
__device__ __forceinline__ void stage_tile_any(const OwnRouteArgs& a, int64_t O,
                                               uint64_t* s_bases, uint64_t* s_hq,
                                               uint64_t* s_bad, uint64_t* s_st) {
  for (int i = threadIdx.x; i < kOwnBaseWords; i += blockDim.x) {
    const int64_t gw = O / 32 + i;
    s_bases[i] = (gw >= 0 && gw < a.base_words) ? a.bases[gw] : 0ull;
  }
  for (int i = threadIdx.x; i < kOwnPlaneWords; i += blockDim.x) {
    const int64_t gw = O / 64 + i;
    const bool in = gw >= 0 && gw < a.plane_words;
    s_hq[i] = in ? a.hq[gw] : 0ull;
    s_bad[i] = in ? a.bad[gw] : ~0ull;
    s_st[i] = in ? a.st[gw] : 0ull;
  }
}

// Level-1 histogram: block b counts the buckets of the windows of routing
// tiles b, b + grid, ... (the tiles the emit kernel gives the same block)
// into column b of the bucket-major matrix h1[bucket * grid + b].
template <int W>
__global__ __launch_bounds__(kOwnRouteThreads) void k_own_hist(OwnRouteArgs a) {
  __shared__ uint64_t s_bases[kOwnBaseWords];
  __shared__ uint64_t s_hq[kOwnPlaneWords];
  __shared__ uint64_t s_bad[kOwnPlaneWords];
  __shared__ uint64_t s_st[kOwnPlaneWords];
  __shared__ uint32_t s_h[kOwnL1Max];
  __shared__ uint64_t s_red[kOwnRouteThreads / 64];
  const int tid = threadIdx.x;
  const int nbins = 1 << a.p1;
  for (int i = tid; i < nbins; i += kOwnRouteThreads) s_h[i] = 0;
  const int koff = 64 * W - 2 * (int)a.k;
  const int64_t n_tiles = (a.n + kOwnTile - 1) / kOwnTile;
  uint64_t nwin = 0;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t P0 = t * kOwnTile, O = P0 - kHalo;
    lds_barrier();
    stage_tile_any(a, O, s_bases, s_hq, s_bad, s_st);
    lds_barrier();
    if (a.shards > 1) {  // the part filter needs the whole key
#pragma unroll 1
      for (int j = 0; j < kOwnTile / kOwnRouteThreads; ++j) {
        uint64_t key[W];
        uint32_t e6;
        if (own_window<W>(s_bases, s_hq, s_bad, s_st, P0 + j * kOwnRouteThreads + tid, O, a.n,
                          a.k, a.shards, a.owner, key, e6)) {
          ++nwin;
          atomicAdd(&s_h[top_bits<W>(key, koff, a.p1)], 1u);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < kOwnTile / kOwnRouteThreads; ++j) {
        const int b = own_top(s_bases, s_bad, s_st, P0 + j * kOwnRouteThreads + tid, O, a.n,
                              a.k, (int)a.p1);
        if (b >= 0) {
          ++nwin;
          atomicAdd(&s_h[b], 1u);
        }
      }
    }
  }
  lds_barrier();
  for (int i = tid; i < nbins; i += kOwnRouteThreads)
    a.h1[(uint64_t)i * gridDim.x + blockIdx.x] = s_h[i];
  block_add(&a.ctr[kCtrWindows], nwin, s_red);
}

// Level-1 emit, staged: the same routing tiles as k_own_hist, taken in
// batches (two tiles for one-word records, else one); a batch's records are
// ranked by bucket in LDS and leave as one contiguous run per bucket at the
// block's cursors (the scanned matrix column), so that HBM sees whole lines
// rather than scattered 8-byte stores.
template <int R>
struct EmitBatch {
  static constexpr int kTiles = R == 1 ? 2 : 1;                  // routing tiles
  static constexpr int kLane = kOwnTile / kOwnRouteThreads;       // windows per lane per tile
  static constexpr int kCap = kTiles * kOwnTile;                  // records per batch
};

template <int W, int R>
__global__ __launch_bounds__(kOwnRouteThreads) void k_own_emit_staged(OwnRouteArgs a) {
  constexpr int BT = EmitBatch<R>::kTiles;
  constexpr int PT = EmitBatch<R>::kLane;
  constexpr int CAP = EmitBatch<R>::kCap;
  __shared__ uint64_t s_bases[kOwnBaseWords];
  __shared__ uint64_t s_hq[kOwnPlaneWords];
  __shared__ uint64_t s_bad[kOwnPlaneWords];
  __shared__ uint64_t s_st[kOwnPlaneWords];
  __shared__ uint64_t s_rec[CAP * R];  // records by window slot (unsorted)
  __shared__ uint16_t s_binr[CAP];     // bucket of each window slot's record (~0: none)
  __shared__ uint16_t s_inv[CAP];      // window slot of each bucket-ordered position
  __shared__ uint32_t s_cnt[kOwnL1Max];
  __shared__ uint32_t s_start[kOwnL1Max];
  __shared__ uint32_t s_cur[kOwnL1Max];
  __shared__ uint32_t s_w[kOwnRouteThreads / 64];
  static_assert(kOwnL1Max <= kOwnRouteThreads, "one bucket per lane in the scan");
  static_assert(CAP <= 65535, "window slots fit 16 bits");
  const int tid = threadIdx.x;
  const int nbins = 1 << a.p1;
  const int roff = 64 * (W + 1) - 2 * (int)a.k - 6;  // the digit in a full record
  const int top_bits_kept = own_rest_bits(a.k) + 6 - 64 * (R - 1);  // 1..64
  const uint64_t top_mask = top_bits_kept >= 64 ? ~0ull : (1ull << top_bits_kept) - 1ull;
  const int64_t G = gridDim.x, blk = blockIdx.x;
  for (int i = tid; i < nbins; i += kOwnRouteThreads) {
    s_cur[i] = a.h1[(uint64_t)i * G + blk];
    s_cnt[i] = 0;
  }
  const int64_t n_tiles = (a.n + kOwnTile - 1) / kOwnTile;
  const int64_t mine = n_tiles > blk ? (n_tiles - blk + G - 1) / G : 0;  // tiles blk + j G
  // The block's tile j is staged as soon as tile j - 1's windows are formed,
  // before the batch's records are written out: one counter tracks a wave's
  // loads and stores alike, so staging after the write-out would wait for
  // every store of the batch to land.
  if (mine > 0) stage_tile_any(a, blk * kOwnTile - kHalo, s_bases, s_hq, s_bad, s_st);
  lds_barrier();
  for (int64_t j0 = 0; j0 < mine; j0 += BT) {
    for (int bt = 0; bt < BT; ++bt) {
      const bool has = j0 + bt < mine;  // uniform over the block
      const int64_t P0 = (blk + (j0 + bt) * G) * kOwnTile, O = P0 - kHalo;
      // a lane's PT consecutive windows, one at a time (its record goes to
      // LDS at once): the first one's words are read from the tile, each
      // next one's shift one base in; the bases shifted in and out are also
      // the windows' neighbours
      const int64_t p0 = P0 + (int64_t)tid * PT;
      const uint32_t lp0 = (uint32_t)(p0 - O);
      const int tb = 2 * (int)a.k - 64 * (W - 1);  // bits of the top word
      uint64_t fw[W], rw[W];
      window_words<W>(s_bases, 2 * lp0, a.k, fw);
      revcomp_words<W>(fw, a.k, rw);
      uint32_t left = get_base(s_bases, lp0 - 1), right = 0;
#pragma unroll 1
      for (int pw = 0; pw < PT; ++pw) {
        const int slot = (bt * PT + pw) * kOwnRouteThreads + tid;
        if (pw > 0) {
          left = (uint32_t)(fw[0] >> (tb - 2)) & 3u;  // the base leaving the window
          roll_words<W>(fw, rw, right, a.k);
        }
        right = get_base(s_bases, lp0 + pw + a.k);  // staged: lp0 + 3 + 127 < kOwnSpan
        uint64_t key[W];
        uint32_t e6 = 0;
        uint16_t b16 = 0xffffu;
        if (has && own_window_fr<W>(s_bases, s_hq, s_bad, s_st, p0 + pw, O, a.n, a.k, a.shards,
                                    a.owner, fw, rw, key, e6, (int)left, (int)right)) {
          uint64_t f[W + 1];
          make_record<W, W + 1>(key, e6, f);
          const uint32_t b = top_bits<W + 1>(f, roff, a.p1);
          // the low R words, without the digit's bits
#pragma unroll
          for (int w = 0; w < R; ++w)
            s_rec[slot * R + w] = w == 0 ? f[W + 1 - R] & top_mask : f[W + 1 - R + w];
          atomicAdd(&s_cnt[b], 1u);
          b16 = (uint16_t)b;
        }
        s_binr[slot] = b16;
      }
      lds_barrier();  // every window of the staged tile is formed
      if (j0 + bt + 1 < mine) {
        const int64_t P1 = (blk + (j0 + bt + 1) * G) * kOwnTile;
        stage_tile_any(a, P1 - kHalo, s_bases, s_hq, s_bad, s_st);
      }
      if (bt + 1 < BT) lds_barrier();  // the batch's next tile is formed next
    }
    uint32_t excl = 0;
    const uint32_t c = tid < nbins ? s_cnt[tid] : 0u;
    const uint32_t total = block_excl_scan(c, excl, s_w);
    if (tid < nbins) {
      s_start[tid] = excl;
      s_cnt[tid] = 0;  // now the fill count of each bucket
    }
    lds_barrier();
    for (int q = 0; q < BT * PT; ++q) {  // bucket-ordered positions of the records
      const int slot = q * kOwnRouteThreads + tid;
      const uint32_t b = s_binr[slot];
      if (b != 0xffffu) s_inv[s_start[b] + atomicAdd(&s_cnt[b], 1u)] = (uint16_t)slot;
    }
    lds_barrier();
    for (uint32_t i = tid; i < total * R; i += kOwnRouteThreads) {
      const uint32_t rr = i / R, w = i - rr * R;
      const uint32_t src = s_inv[rr], b = s_binr[src];
      a.rec[((uint64_t)s_cur[b] + (rr - s_start[b])) * R + w] = s_rec[src * R + w];
    }
    lds_barrier();
    if (tid < nbins) {
      s_cur[tid] += c;
      s_cnt[tid] = 0;
    }
    lds_barrier();  // the next batch counts into s_cnt at once
  }
}

// ------------------------------------------------------ level 2 route ----

// Records per level-2 chunk (one block): 8,192 record words.
template <int R>
struct PartShape {
  static constexpr int kChunk = R == 1 ? 8192 : (R == 2 ? 4096 : (R <= 4 ? 2048 : 1024));
  static constexpr int kPerThread = kChunk / kOwnPartThreads;
};

int own_chunk_records(uint32_t k) {
  const int R = own_record_words(k);
  return R == 1 ? 8192 : (R == 2 ? 4096 : (R <= 4 ? 2048 : 1024));
}

// The bucket of every owner and of every level-2 chunk (one block per
// bucket), so that later kernels find theirs with one load.
__global__ void k_own_maps(OwnPartArgs a) {
  const OwnBucket bk = a.buckets[blockIdx.x];
  const uint32_t n_own = 1u << bk.p2;
  for (uint32_t i = threadIdx.x; i < n_own; i += blockDim.x) {
    a.owner_bucket[bk.sbbase + i] = (uint16_t)blockIdx.x;
    a.owner_pfx[bk.sbbase + i] = (uint8_t)(a.p1 + bk.p2);
  }
  for (uint32_t i = threadIdx.x; i < bk.chunks; i += blockDim.x)
    a.chunk_bucket[bk.cbase + i] = (uint16_t)blockIdx.x;
}

// Level-2 histogram: chunk c of bucket b counts its records' next p2_b key
// bits into its row of the bucket's chunk-major matrix,
// m[b.mbase + c * 2^p2_b + digit].
template <int R>
__global__ __launch_bounds__(kOwnPartThreads) void k_own_hist2(OwnPartArgs a) {
  __shared__ uint32_t s_h[1 << kOwnL2Max];
  constexpr int CH = PartShape<R>::kChunk;
  const int tid = threadIdx.x;
  const int b = a.chunk_bucket[blockIdx.x];
  const OwnBucket bk = a.buckets[b];
  const uint32_t c = blockIdx.x - bk.cbase;
  const int nbins = 1 << bk.p2;
  for (int i = tid; i < nbins; i += kOwnPartThreads) s_h[i] = 0;
  lds_barrier();
  const uint64_t r0 = bk.start + (uint64_t)c * CH;
  const uint64_t r1 = r0 + (uint64_t)CH < bk.start + bk.n ? r0 + (uint64_t)CH : bk.start + bk.n;
  const int roff = 64 * R - 2 * (int)a.k - 6 + (int)a.p1;
  for (uint64_t r = r0 + tid; r < r1; r += kOwnPartThreads) {
    uint64_t v[R];
    load_record<R>(a.rec_in, r, v);
    atomicAdd(&s_h[top_bits<R>(v, roff, (int)bk.p2)], 1u);
  }
  lds_barrier();
  for (int i = tid; i < nbins; i += kOwnPartThreads)
    a.m[bk.mbase + (uint64_t)c * nbins + i] = s_h[i];
}

// Level-2 scatter: the same chunks, ranked by digit in LDS and written as
// one run per owner at the chunk's cursors (owner start + the column prefix
// of the matrix).
template <int R>
__global__ __launch_bounds__(kOwnPartThreads) void k_own_scatter2(OwnPartArgs a) {
  constexpr int CH = PartShape<R>::kChunk;
  constexpr int PT = PartShape<R>::kPerThread;
  __shared__ uint64_t s_rec[CH * R];
  __shared__ uint16_t s_bin[CH];
  __shared__ uint32_t s_cnt[1 << kOwnL2Max];
  __shared__ uint32_t s_start[1 << kOwnL2Max];
  __shared__ uint32_t s_cur[1 << kOwnL2Max];
  __shared__ uint32_t s_w[kOwnPartThreads / 64];
  const int tid = threadIdx.x;
  const int b = a.chunk_bucket[blockIdx.x];
  const OwnBucket bk = a.buckets[b];
  const uint32_t c = blockIdx.x - bk.cbase;
  const int nbins = 1 << bk.p2;
  for (int i = tid; i < nbins; i += kOwnPartThreads) {
    s_cnt[i] = 0;
    s_cur[i] = a.start2[bk.sbbase + i] + a.m[bk.mbase + (uint64_t)c * nbins + i];
  }
  lds_barrier();
  const uint64_t r0 = bk.start + (uint64_t)c * CH;
  const uint64_t r1 = r0 + (uint64_t)CH < bk.start + bk.n ? r0 + (uint64_t)CH : bk.start + bk.n;
  const int roff = 64 * R - 2 * (int)a.k - 6 + (int)a.p1;
  uint64_t v[PT][R];
  uint32_t bin[PT], rank[PT];
#pragma unroll
  for (int q = 0; q < PT; ++q) {
    const uint64_t r = r0 + (uint64_t)q * kOwnPartThreads + tid;
    bin[q] = 0xffffffffu;
    rank[q] = 0;
#pragma unroll
    for (int w = 0; w < R; ++w) v[q][w] = 0;
    if (r < r1) load_record<R>(a.rec_in, r, v[q]);
  }
#pragma unroll
  for (int q = 0; q < PT; ++q) {
    const uint64_t r = r0 + (uint64_t)q * kOwnPartThreads + tid;
    if (r < r1) {
      bin[q] = top_bits<R>(v[q], roff, (int)bk.p2);
      rank[q] = atomicAdd(&s_cnt[bin[q]], 1u);
    }
  }
  lds_barrier();
  // bucket starts: nbins <= 2 * kOwnPartThreads values, two per thread
  const uint32_t c0 = 2 * tid < nbins ? s_cnt[2 * tid] : 0u;
  const uint32_t c1 = 2 * tid + 1 < nbins ? s_cnt[2 * tid + 1] : 0u;
  uint32_t excl = 0;
  block_excl_scan(c0 + c1, excl, s_w);
  if (2 * tid < nbins) s_start[2 * tid] = excl;
  if (2 * tid + 1 < nbins) s_start[2 * tid + 1] = excl + c0;
  lds_barrier();
#pragma unroll
  for (int q = 0; q < PT; ++q) {
    if (bin[q] == 0xffffffffu) continue;
    const uint32_t pos = s_start[bin[q]] + rank[q];
#pragma unroll
    for (int w = 0; w < R; ++w) s_rec[pos * R + w] = v[q][w];
    s_bin[pos] = (uint16_t)bin[q];
  }
  lds_barrier();
  const uint32_t n = (uint32_t)(r1 - r0);
  for (uint32_t i = tid; i < n * R; i += kOwnPartThreads) {
    const uint32_t rr = i / R, d = s_bin[rr];
    a.rec_out[((uint64_t)s_cur[d] + (rr - s_start[d])) * R + (i - rr * R)] = s_rec[i];
  }
}

// Column scan of the level-2 matrix: one thread per owner (bucket b, digit
// d) turns its column (chunks 0, 1, ... of b) into exclusive prefixes and
// leaves the owner's record count in tot[owner]; thread n_owners writes 0, so
// that an exclusive scan of tot[0 .. n_owners] gives every owner's first
// record and the total after the last.
__global__ void k_own_colscan(OwnPartArgs a, uint32_t n_owners) {
  const uint32_t sb = blockIdx.x * blockDim.x + threadIdx.x;
  if (sb > n_owners) return;
  if (sb == n_owners) {
    a.start2[sb] = 0;
    return;
  }
  const int b = a.owner_bucket[sb];
  const OwnBucket bk = a.buckets[b];
  const uint32_t d = sb - bk.sbbase, nbins = 1u << bk.p2;
  uint32_t run = 0;
  for (uint32_t c = 0; c < bk.chunks; ++c) {
    const uint64_t i = bk.mbase + (uint64_t)c * nbins + d;
    const uint32_t v = a.m[i];
    a.m[i] = run;
    run += v;
  }
  a.start2[sb] = run;
}

// ------------------------------------------------------------- owners ----

// LDS table slots per owner: as many as fit (a multiple of 64) beside the
// Bloom filter in one owner block's share of the CU's
// 160 KiB (kOwnBlocksPerCU blocks share a CU), and at most kRecLanes x
// threads / 2, so that an owner's 2T records are kRecLanes per lane: more
// records per lane spill registers at four waves per SIMD.
template <int C>
struct OwnerShape {
  static constexpr int kPerSlot = 8 * C + 4 + 32 + 2;  // chunks, count, tallies, row list
  static constexpr int kFixed = kOwnBloomWords * 8 + 16 + 8 + (kOwnThreads / 64) * 4 * 5 + 256;
  static constexpr int kFit = (kOwnLdsBytes - kFixed) / kPerSlot / 64 * 64;
  static constexpr int kRecLanes = C == 1 ? 5 : (C <= 3 ? 4 : 3);
  static constexpr int kCap = kRecLanes * kOwnThreads / 2;
  static constexpr int kSlots = kFit < kCap ? kFit : kCap;
  static_assert(kFixed + kSlots * kPerSlot <= kOwnLdsBytes, "owner LDS");
};


int own_slots(uint32_t k) {
  switch (own_chunks(k)) {
    case 1: return OwnerShape<1>::kSlots;
    case 2: return OwnerShape<2>::kSlots;
    case 3: return OwnerShape<3>::kSlots;
    case 4: return OwnerShape<4>::kSlots;
    default: return OwnerShape<5>::kSlots;
  }
}

// One owner per block: Bloom pass A and count pass B over the owner's
// records in LDS, then classify (count >= min_count, extension codes), sort
// by key and write the rows to the owner's staging rows.
template <int R, int C>
__global__ __launch_bounds__(kOwnThreads, kOwnThreads * kOwnBlocksPerCU / 256) void k_own_count(OwnCountArgs a) {
  constexpr int T = OwnerShape<C>::kSlots;
  // records per lane per batch: an owner of the usual size (up to 2 T
  // records) is one batch
  constexpr int NB = (2 * T + kOwnThreads - 1) / kOwnThreads;
  constexpr uint64_t kBatch = (uint64_t)NB * kOwnThreads;
  __shared__ uint64_t s_bloom[kOwnBloomWords];
  __shared__ uint64_t s_ch[C][T];
  __shared__ uint32_t s_cnt[T];  // occurrences without a left extension
  __shared__ uint32_t s_tal[8][T];
  __shared__ uint16_t s_list[T];  // the owner's kept slots, in slot order
  __shared__ uint32_t s_misc[4];
  __shared__ uint64_t s_chunk;
  __shared__ uint32_t s_w[kOwnThreads / 64];
  __shared__ uint32_t s_acc[4];  // the owner's first sightings, second, passed, claimed
  const int tid = threadIdx.x;
  const uint32_t k = a.k;
  constexpr int ws = C;  // the launcher picks C = own_chunks(k)
  const int W = (int)(k + 31) / 32;
  const uint32_t tcap = a.slots < (uint32_t)T ? a.slots : (uint32_t)T;
  const uint32_t N = a.n_owners, G = gridDim.x;
  // optional phase clocks (thread 0, summed over the block's owners)
  uint64_t prof_acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  uint64_t prof_t = 0;
#define PROF_MARK(e)                                         \
  if (a.prof && tid == 0) {                                  \
    const uint64_t now_ = wall_clock64();                    \
    if ((e) > 0) prof_acc[(e) > 8 ? 7 : ((e) > 0 ? (e) - 1 : 0)] += now_ - prof_t; \
    prof_t = now_;                                           \
  }

  // Persistent blocks: owners sb = blockIdx.x, + G, ...
  uint64_t st_cur = 0, st_end = 0;  // the block's staging chunk (uniform)
  for (uint32_t sb = blockIdx.x; sb < N; sb += G) {
  const uint64_t r0 = a.start2[sb], r1 = a.start2[sb + 1];
  // an owner of at most NB records per lane is loaded once for both passes
  const bool one_batch = r1 - r0 <= kBatch;
  uint64_t vb[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const uint64_t r = r0 + (uint64_t)q * kOwnThreads + tid;
#pragma unroll
    for (int w = 0; w < R; ++w) vb[q][w] = 0;
    if (one_batch && r < r1) load_record<R>(a.rec, r, vb[q]);
  }

  PROF_MARK(0);
  for (int i = tid; i < kOwnBloomWords; i += kOwnThreads) s_bloom[i] = 0;
  for (int i = tid; i < T; i += kOwnThreads) {
#pragma unroll
    for (int c = 0; c < C; ++c) s_ch[c][i] = 0;
    s_cnt[i] = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) s_tal[e][i] = 0;
  }
  if (tid == 0) {
    s_misc[0] = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) s_acc[e] = 0;
  }
  lds_barrier();
  PROF_MARK(1);

  uint32_t l1 = 0, l2 = 0, passed = 0, claimed = 0;
  // Both passes take a lane's records of a batch together, one memory step
  // at a time for all of them (hashes, then every LDS load, then every
  // atomic), so a lane has several LDS round trips in flight instead of one.
  // ---- pass A (Bloom): every sighting sets the key's level-1 pattern; a
  // sighting of a key whose level-1 pattern was complete completes level 2
  if (a.use_bloom) {
    for (uint64_t b0 = r0; b0 < r1; b0 += kBatch) {
      // this lane's records of the batch are its first nq
      const int nq = lane_records<NB>(b0, r1, tid);
      uint32_t bi[NB], pat[NB];
      uint64_t cur[NB];
      if (!one_batch) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {  // every load of the batch in flight at once
#pragma unroll
          for (int w = 0; w < R; ++w) vb[q][w] = 0;
          if (q < nq) load_record<R>(a.rec, b0 + (uint64_t)q * kOwnThreads + tid, vb[q]);
        }
      }
      // hashes of every slot (a slot past the owner's records holds zeros):
      // no branch per record
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        uint64_t key[R], ch[C];
        record_key<R>(vb[q], key);
        to_chunks<R, C>(key, ws, ch);
        owner_bloom(owner_hash<C>(ch, ws), bi[q], pat[q]);
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) cur[q] = s_bloom[bi[q]];
      bool set1[NB], set2[NB];
      uint64_t old[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        set1[q] = q < nq && ((uint32_t)cur[q] & pat[q]) != pat[q];
        set2[q] = q < nq && !set1[q] && ((uint32_t)(cur[q] >> 32) & pat[q]) != pat[q];
        old[q] = 0;
        if (set1[q] || set2[q])
          old[q] = atomicOr(reinterpret_cast<unsigned long long*>(&s_bloom[bi[q]]),
                            set1[q] ? (unsigned long long)pat[q]
                                    : (unsigned long long)pat[q] << 32);
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (set1[q]) {
          if (((uint32_t)old[q] & pat[q]) != pat[q]) {
            ++l1;  // first sighting (up to false positives)
          } else {  // seen meanwhile: complete the level-2 pattern
            const uint64_t o2 = atomicOr(reinterpret_cast<unsigned long long*>(&s_bloom[bi[q]]),
                                         (unsigned long long)pat[q] << 32);
            if (((uint32_t)(o2 >> 32) & pat[q]) != pat[q]) ++l2;
          }
        } else if (set2[q] && ((uint32_t)(old[q] >> 32) & pat[q]) != pat[q]) {
          ++l2;
        }
      }
    }
    lds_barrier();
  }
  PROF_MARK(2);
  // ---- pass B: count the records whose key completed level 2 (all records
  // without the Bloom screen) in the open-addressing LDS table.  Each stored
  // chunk is written once by CAS from 0 (chunks never are 0), so a slot's
  // chunks always spell one key and equal keys meet in one slot (a word
  // read as 0 may have been written since, which the CAS then reports; a
  // non-zero word is final).  An occurrence adds 1 to its left tally (or to the no-left-extension count)
  // and 1 to its right tally if it has one: the count is the sum of the
  // first five, so it needs no add of its own.
  for (uint64_t b0 = r0; b0 < r1; b0 += kBatch) {
    const int nq = lane_records<NB>(b0, r1, tid);
    uint32_t okm = (1u << nq) - 1u;  // bit q: record q is counted
    uint64_t ch[NB][C], w0[NB], h[NB];
    uint32_t i0[NB];
    if (!one_batch) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
#pragma unroll
        for (int w = 0; w < R; ++w) vb[q][w] = 0;
        if (q < nq) load_record<R>(a.rec, b0 + (uint64_t)q * kOwnThreads + tid, vb[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      uint64_t key[R];
      record_key<R>(vb[q], key);
      to_chunks<R, C>(key, ws, ch[q]);
      h[q] = owner_hash<C>(ch[q], ws);
    }
    if (a.use_bloom) {
      uint32_t bi[NB], pat[NB];
      uint64_t bw[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) owner_bloom(h[q], bi[q], pat[q]);
#pragma unroll
      for (int q = 0; q < NB; ++q) bw[q] = s_bloom[bi[q]];
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (((uint32_t)(bw[q] >> 32) & pat[q]) != pat[q]) okm &= ~(1u << q);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {  // first word of every record's first probe at once
      i0[q] = __umulhi((uint32_t)(h[q] >> 32), tcap);
      w0[q] = s_ch[0][i0[q]];
    }
    int slot[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      slot[q] = -1;
      if (!((okm >> q) & 1u)) continue;
      ++passed;
      uint32_t i = i0[q];
      for (uint32_t probe = 0; probe < tcap; ++probe) {
        bool match = true;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          if (c < ws && match) {
            uint64_t w = (probe == 0 && c == 0) ? w0[q] : s_ch[c][i];
            if (w == 0) {
              const uint64_t o = atomicCAS(reinterpret_cast<unsigned long long*>(&s_ch[c][i]),
                                           0ull, (unsigned long long)ch[q][c]);
              w = o == 0 ? ch[q][c] : o;
              if (o == 0 && c == 0) ++claimed;
            }
            match = w == ch[q][c];
          }
        }
        if (match) {
          slot[q] = (int)i;
          break;
        }
        if (++i == tcap) i = 0;
      }
      if (slot[q] < 0) s_misc[0] = 1;  // the owner's keys do not fit: split finer
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (slot[q] < 0) continue;
      const uint32_t e6 = (uint32_t)(vb[q][R - 1] & 63u);
      atomicAdd((e6 & 32u) ? &s_tal[(e6 >> 3) & 3u][slot[q]] : &s_cnt[slot[q]], 1u);
      if (e6 & 4u) atomicAdd(&s_tal[4 + (e6 & 3u)][slot[q]], 1u);
    }
  }
  // ---- statistics, added once per owner to one of kOwnStripes copies of
  // the counters (the host sums them): each wave adds its sums into LDS, and
  // the barrier that completes the table also completes them
  PROF_MARK(3);
  unsigned long long* sc = a.ctr + (uint64_t)(sb % kOwnStripes) * kCtrCount;
  {
    uint32_t v[4] = {l1, l2, passed, claimed};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      for (int o = 32; o > 0; o >>= 1) v[e] += __shfl_down(v[e], o);
    if ((tid & 63) == 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (v[e]) atomicAdd(&s_acc[e], v[e]);
    }
  }
  lds_barrier();
  // s_misc[0] and s_acc change only in the next owner's clear, after a
  // barrier every lane passes after reading them
  const bool overflow = s_misc[0] != 0;
  if (tid == 0) {
    const uint32_t t0 = s_acc[0], t1 = s_acc[1], t2 = s_acc[2], t3 = s_acc[3];
    if (t0) atomicAdd(&sc[kCtrL1New], (unsigned long long)t0);
    if (t1) atomicAdd(&sc[kCtrL2New], (unsigned long long)t1);
    if (t2) atomicAdd(&sc[kCtrPassed], (unsigned long long)t2);
    if (t3) atomicAdd(&sc[kCtrClaimed], (unsigned long long)t3);
    // keys of the fullest owner, and the owners whose keys did not fit
    atomicMax(&sc[kCtrWindows], (unsigned long long)t3);
    if (overflow) {
      atomicAdd(&sc[kCtrHeavy], 1ull);
      atomicOr(&sc[kCtrStatus], (unsigned long long)kStatusProbeLimit);
    }
  }
  if (overflow) {  // uniform: the flag is stable until the barrier below
    if (tid == 0) {
      a.rows_sb[sb] = 0;
      a.row_off[sb] = 0;
    }
    lds_barrier();  // every lane has read the flag and tid 0 the sums
    continue;
  }

  PROF_MARK(4);
  // ---- classify: a slot is a row when its count reaches min_count.  Rows
  // leave in slot order, each thread's at its place from one block scan;
  // the copy to the table puts every owner's rows in key order.
  // Rows are ranked in slot order (slot i = tid + m x kOwnThreads): one scan
  // of the kept flags of every m at once, packed in 11-bit fields (each m's
  // count is at most kOwnThreads); the kept slots are then listed in LDS so
  // that every lane writes the same number of rows.
  constexpr int SP = (T + kOwnThreads - 1) / kOwnThreads;  // slots per thread
  static_assert(SP <= 3 && (SP < 3 || T - 2 * kOwnThreads < 1024), "packed rank fields");
  uint32_t keep = 0, packed = 0;
#pragma unroll
  for (int m = 0; m < SP; ++m) {
    const uint32_t i = tid + m * kOwnThreads;
    if (i < tcap && s_ch[0][i] != 0 &&
        s_cnt[i] + s_tal[0][i] + s_tal[1][i] + s_tal[2][i] + s_tal[3][i] >= a.min_count) {
      keep |= 1u << m;
      packed += 1u << (11 * m);
    }
  }
  PROF_MARK(5);
  uint32_t excl_p = 0;
  const uint32_t total_p = block_excl_scan(packed, excl_p, s_w);
  uint32_t first[SP];  // first row of slot column m
  uint32_t rows = 0;
#pragma unroll
  for (int m = 0; m < SP; ++m) {
    first[m] = rows + ((excl_p >> (11 * m)) & 0x7ffu);
    rows += (total_p >> (11 * m)) & 0x7ffu;
  }
#pragma unroll
  for (int m = 0; m < SP; ++m)  // the kept slots in slot order
    if ((keep >> m) & 1u) s_list[first[m]] = (uint16_t)(tid + m * kOwnThreads);
  lds_barrier();
  PROF_MARK(6);
  PROF_MARK(7);
  // ---- rows to staging.  Blocks take chunks of staging
  // rows from a shared cursor (one atomic per chunk, not per owner) and fill
  // them owner after owner; an owner past the end of staging is flagged and
  // the pass runs again with every owner's rows at its scanned offset.
  uint64_t base;
  bool fits = true;
  if (a.st_fixed) {
    base = a.st_fixed[sb];
  } else {
    if (st_cur + rows > st_end) {  // uniform
      const uint64_t want = rows > a.st_chunk ? rows : a.st_chunk;
      if (tid == 0) s_chunk = atomicAdd(a.st_cursor, (unsigned long long)want);
      lds_barrier();
      st_cur = s_chunk;
      st_end = st_cur + want;
    }
    base = st_cur;
    fits = base + rows <= a.st_cap;
    st_cur += rows;
  }
  // the key's level-1 digit goes back above its rest bits
  const uint64_t digit = a.owner_bucket[sb];
  const int rest_bits = own_rest_bits(k), dw = rest_bits >> 6, doff = rest_bits & 63;
  for (uint32_t j = tid; j < (fits ? rows : 0u); j += kOwnThreads) {
    const uint32_t i = s_list[j];
    uint64_t cv[C], f[R];
#pragma unroll
    for (int c = 0; c < C; ++c) cv[c] = s_ch[c][i];
    from_chunks<R>(cv, ws, f);
    const uint64_t row = base + j;
    uint64_t lw[R + 1];  // the whole key (W <= R + 1 words), least significant first
#pragma unroll
    for (int q = 0; q <= R; ++q) {
      lw[q] = q < R ? f[R - 1 - q] : 0ull;
      if (q == dw) lw[q] |= digit << doff;
      if (q == dw + 1 && doff > 0) lw[q] |= digit >> (64 - doff);
    }
#pragma unroll
    for (int q = 0; q <= R; ++q)
      if (q < W) a.st_keys[row * W + (W - 1 - q)] = lw[q];
    uint32_t l[4], rr[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      l[e] = s_tal[e][i];
      rr[e] = s_tal[4 + e][i];
    }
    const uint32_t cnt = s_cnt[i] + l[0] + l[1] + l[2] + l[3];
    a.st_counts[row] = cnt;
    uint4* ep = reinterpret_cast<uint4*>(a.st_ext + row * 8);
    ep[0] = make_uint4(l[0], l[1], l[2], l[3]);
    ep[1] = make_uint4(rr[0], rr[1], rr[2], rr[3]);
    reinterpret_cast<uint16_t*>(a.st_codes)[row] =
        (uint16_t)((uint32_t)side_code(l, cnt, a.t_min_ext, a.t_base, a.err_ppm) |
                   ((uint32_t)side_code(rr, cnt, a.t_min_ext, a.t_base, a.err_ppm) << 8));
  }
  if (tid == 0) {
    a.rows_sb[sb] = rows;
    a.row_off[sb] = rows;
    a.st_off[sb] = base;
    if (rows) atomicAdd(&sc[kCtrRows], (unsigned long long)rows);
    if (!fits) atomicOr(&sc[kCtrStatus], (unsigned long long)kStatusStaging);
  }
  lds_barrier();  // the rows have left LDS: the next owner may clear it
  PROF_MARK(8);
  }
  if (a.prof && tid == 0)
    for (int e = 0; e < 8; ++e) atomicAdd(&a.prof[e], (unsigned long long)prof_acc[e]);
#undef PROF_MARK
}

// Owners' rows from staging to the table at the scanned row offsets, in key
// order (one block per owner; the owner pass leaves them in slot order).
// The owner's keys share its prefix, so each row's sort key is the next
// (at most) 32 key bits: rows are bucketed by the top kOwnSortBits of them,
// each bucket (almost always 0-2 rows) is ordered by them (by the whole key,
// read again, when two are equal), and every row is copied to its place.
// NR: rows of an owner at most for W-word keys.
template <int W, int NR>
__global__ __launch_bounds__(kOwnCopyThreads) void k_own_copy(OwnCopyArgs a) {
  constexpr int NSB = 1 << kOwnSortBits;
  __shared__ uint32_t s_k32[NR];
  __shared__ uint16_t s_rank[NR];
  __shared__ uint16_t s_ord[NR];
  __shared__ uint32_t s_bc[NSB];
  __shared__ uint32_t s_bs[NSB];
  __shared__ uint32_t s_w[kOwnCopyThreads / 64];
  const int tid = threadIdx.x;
  const uint32_t sb = blockIdx.x;
  const uint32_t n = a.rows_sb[sb];
  if (n == 0) return;  // the whole block
  const uint64_t src0 = a.st_off[sb], dst0 = a.row_off[sb];
  const int pfx = a.owner_pfx[sb];
  const int rest = 2 * (int)a.k - pfx;
  const int len = rest < 32 ? (rest > 0 ? rest : 0) : 32;  // sort-key bits
  const int nb = len < kOwnSortBits ? len : kOwnSortBits;
  const int nbins = 1 << nb;
  const int koff = 64 * W - 2 * (int)a.k + pfx;
  for (int i = tid; i < nbins; i += kOwnCopyThreads) s_bc[i] = 0;
  lds_barrier();
  for (uint32_t r = tid; r < n; r += kOwnCopyThreads) {
    uint64_t v[W];
#pragma unroll
    for (int w = 0; w < W; ++w) v[w] = a.st_keys[(src0 + r) * W + w];
    const uint32_t x = top_bits<W>(v, koff, len);
    s_k32[r] = x;
    s_rank[r] = (uint16_t)atomicAdd(&s_bc[x >> (len - nb)], 1u);
  }
  lds_barrier();
  // bucket starts: NSB / kOwnCopyThreads consecutive buckets per thread
  constexpr int BPT = NSB / kOwnCopyThreads;
  uint32_t mine = 0;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int d = tid * BPT + q;
    mine += d < nbins ? s_bc[d] : 0u;
  }
  uint32_t excl = 0;
  block_excl_scan(mine, excl, s_w);
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int d = tid * BPT + q;
    if (d < nbins) {
      s_bs[d] = excl;
      excl += s_bc[d];
    }
  }
  lds_barrier();
  for (uint32_t r = tid; r < n; r += kOwnCopyThreads)
    s_ord[s_bs[s_k32[r] >> (len - nb)] + s_rank[r]] = (uint16_t)r;
  lds_barrier();
  for (int d = tid; d < nbins; d += kOwnCopyThreads) {  // insertion sort of each bucket
    const uint32_t cnt = s_bc[d], st = s_bs[d];
    for (uint32_t x = st + 1; x < st + cnt; ++x) {
      const uint16_t cur = s_ord[x];
      const uint32_t kc = s_k32[cur];
      int y = (int)x - 1;
      while (y >= (int)st) {
        const uint16_t o = s_ord[y];
        const uint32_t ko = s_k32[o];
        bool less = kc < ko;
        if (kc == ko) {  // the next bits decide (most significant word first)
          for (int w = 0; w < W; ++w) {
            const uint64_t p = a.st_keys[(src0 + cur) * W + w];
            const uint64_t q = a.st_keys[(src0 + o) * W + w];
            if (p != q) {
              less = p < q;
              break;
            }
          }
        }
        if (!less) break;
        s_ord[y + 1] = o;
        --y;
      }
      s_ord[y + 1] = cur;
    }
  }
  lds_barrier();
  for (uint32_t j = tid; j < n; j += kOwnCopyThreads) {
    const uint64_t s = src0 + s_ord[j], d = dst0 + j;
#pragma unroll
    for (int w = 0; w < W; ++w) a.keys[d * W + w] = a.st_keys[s * W + w];
    a.counts[d] = a.st_counts[s];
    const uint4* se = reinterpret_cast<const uint4*>(a.st_ext + s * 8);
    uint4* de = reinterpret_cast<uint4*>(a.ext + d * 8);
    de[0] = se[0];
    de[1] = se[1];
    reinterpret_cast<uint16_t*>(a.codes)[d] = reinterpret_cast<const uint16_t*>(a.st_codes)[s];
  }
}

// dst[i] = src[i * stride], i < n (the first column of a histogram matrix).
__global__ void k_gather_strided(const uint32_t* __restrict__ src, uint64_t stride, uint32_t n,
                                 uint32_t* __restrict__ dst) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[(uint64_t)i * stride];
}

// ---------------------------------------------------------- launchers ----

void launch_gather_strided(const uint32_t* src, uint64_t stride, uint32_t n, uint32_t* dst,
                           hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather_strided, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     src, stride, n, dst);
}

void launch_own_hist(const OwnRouteArgs& a, int grid, hipStream_t s) {
  const dim3 g(grid), t(kOwnRouteThreads);
  switch ((a.k + 31) / 32) {
    case 1: hipLaunchKernelGGL(k_own_hist<1>, g, t, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_own_hist<2>, g, t, 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_own_hist<3>, g, t, 0, s, a); break;
    default: hipLaunchKernelGGL(k_own_hist<4>, g, t, 0, s, a); break;
  }
}

void launch_own_emit(const OwnRouteArgs& a, int grid, hipStream_t s) {
  const int W = (int)(a.k + 31) / 32;
  const int R = own_record_words(a.k);  // W - 1 .. W words
  const dim3 g(grid), t(kOwnRouteThreads);
  if (W == 1) hipLaunchKernelGGL((k_own_emit_staged<1, 1>), g, t, 0, s, a);
  else if (W == 2 && R == 1) hipLaunchKernelGGL((k_own_emit_staged<2, 1>), g, t, 0, s, a);
  else if (W == 2) hipLaunchKernelGGL((k_own_emit_staged<2, 2>), g, t, 0, s, a);
  else if (W == 3 && R == 2) hipLaunchKernelGGL((k_own_emit_staged<3, 2>), g, t, 0, s, a);
  else if (W == 3) hipLaunchKernelGGL((k_own_emit_staged<3, 3>), g, t, 0, s, a);
  else if (R == 3) hipLaunchKernelGGL((k_own_emit_staged<4, 3>), g, t, 0, s, a);
  else hipLaunchKernelGGL((k_own_emit_staged<4, 4>), g, t, 0, s, a);
}

void launch_own_part(const OwnPartArgs& a, uint32_t n_chunks, int scatter, hipStream_t s) {
  if (n_chunks == 0) return;
  const int R = own_record_words(a.k);  // 1 .. 4
  const dim3 g(n_chunks), t(kOwnPartThreads);
  if (!scatter) {
    switch (R) {
      case 1: hipLaunchKernelGGL(k_own_hist2<1>, g, t, 0, s, a); break;
      case 2: hipLaunchKernelGGL(k_own_hist2<2>, g, t, 0, s, a); break;
      case 3: hipLaunchKernelGGL(k_own_hist2<3>, g, t, 0, s, a); break;
      default: hipLaunchKernelGGL(k_own_hist2<4>, g, t, 0, s, a); break;
    }
  } else {
    switch (R) {
      case 1: hipLaunchKernelGGL(k_own_scatter2<1>, g, t, 0, s, a); break;
      case 2: hipLaunchKernelGGL(k_own_scatter2<2>, g, t, 0, s, a); break;
      case 3: hipLaunchKernelGGL(k_own_scatter2<3>, g, t, 0, s, a); break;
      default: hipLaunchKernelGGL(k_own_scatter2<4>, g, t, 0, s, a); break;
    }
  }
}

void launch_own_maps(const OwnPartArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_own_maps, dim3(a.n_buckets), dim3(kBlock), 0, s, a);
}

void launch_own_colscan(const OwnPartArgs& a, uint32_t n_owners, hipStream_t s) {
  const uint32_t n = n_owners + 1;
  hipLaunchKernelGGL(k_own_colscan, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a,
                     n_owners);
}

void launch_own_count(const OwnCountArgs& a, uint32_t blocks, hipStream_t s) {
  if (a.n_owners == 0) return;
  const int R = own_record_words(a.k);
  const int C = own_chunks(a.k);  // R - 1 .. R chunks (rest bits + 6 over 64, rest over 62)
  const dim3 g(blocks < a.n_owners ? blocks : a.n_owners), t(kOwnThreads);
  if (R == 1) hipLaunchKernelGGL((k_own_count<1, 1>), g, t, 0, s, a);
  else if (R == 2 && C == 1) hipLaunchKernelGGL((k_own_count<2, 1>), g, t, 0, s, a);
  else if (R == 2) hipLaunchKernelGGL((k_own_count<2, 2>), g, t, 0, s, a);
  else if (R == 3 && C == 2) hipLaunchKernelGGL((k_own_count<3, 2>), g, t, 0, s, a);
  else if (R == 3) hipLaunchKernelGGL((k_own_count<3, 3>), g, t, 0, s, a);
  else hipLaunchKernelGGL((k_own_count<4, 4>), g, t, 0, s, a);
}

void launch_own_copy(const OwnCopyArgs& a, uint32_t n_owners, hipStream_t s) {
  if (n_owners == 0) return;
  // rows of an owner at most: the slots of the fewest key chunks a W-word
  // key can have (W = 1, 2: one chunk; 3: two; 4: three)
  const dim3 g(n_owners), t(kOwnCopyThreads);
  switch (a.W) {
    case 1: hipLaunchKernelGGL((k_own_copy<1, OwnerShape<1>::kSlots>), g, t, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_own_copy<2, OwnerShape<1>::kSlots>), g, t, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_own_copy<3, OwnerShape<2>::kSlots>), g, t, 0, s, a); break;
    default: hipLaunchKernelGGL((k_own_copy<4, OwnerShape<3>::kSlots>), g, t, 0, s, a); break;
  }
}

}  // namespace kh
