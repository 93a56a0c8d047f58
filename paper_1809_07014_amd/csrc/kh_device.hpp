// Device helpers shared by the k-mer kernels (gfx950, wave64).
//
// Data layout in HBM (all arrays are indexed by the global base position p of
// the concatenated reads):
//   bases  2 bits per base, 32 bases per uint64, most significant pair first
//          (A=0, C=1, G=2, T=3).  Reading bits MSB-first therefore reads the
//          bases in order, and any run of k bases is a 2k-bit integer whose
//          numeric order is the lexicographic order of the k-mer.
//   hq     1 bit per base, 64 per uint64, MSB-first: the base is A/C/G/T and
//          its Phred score reaches the quality cutoff.
//   bad    1 bit per base: the byte is not A/C/G/T.
//   st     1 bit per base: a read starts here.
// A window starting at p is a k-mer iff p + k <= n, no bad bit lies in
// [p, p+k) and no read starts in (p, p+k).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kh {

constexpr int kBlock = 256;             // threads per block (4 waves)
constexpr int kTile = 1024;             // window starts per tile
constexpr int kHalo = 64;               // positions staged before the tile
constexpr int kSpan = kTile + 256;      // staged positions (tile + halos, k <= 127)
constexpr int kBaseWords = kSpan / 32 + 1;
constexpr int kPlaneWords = kSpan / 64 + 1;

// ---- bit access (MSB-first) ------------------------------------------------

// Bits [pos, pos+len) of an MSB-first bit string, right-aligned; 1 <= len <= 64.
__device__ __forceinline__ uint64_t get_bits(const uint64_t* w, uint32_t pos,
                                             uint32_t len) {
  const uint32_t q = pos >> 6, r = pos & 63;
  uint64_t hi = w[q] << r;
  if (r) hi |= w[q + 1] >> (64 - r);
  return len >= 64 ? hi : hi >> (64 - len);
}

// Is any bit set in [pos, pos+len)?  0 <= len <= 128.
__device__ __forceinline__ bool any_bits(const uint64_t* w, uint32_t pos,
                                         uint32_t len) {
  uint64_t acc = 0;
  if (len > 64) {
    acc = get_bits(w, pos, 64);
    pos += 64;
    len -= 64;
  }
  if (len > 0) acc |= get_bits(w, pos, len);
  return acc != 0;
}

__device__ __forceinline__ uint32_t get_bit(const uint64_t* w, uint32_t pos) {
  return (uint32_t)(w[pos >> 6] >> (63 - (pos & 63))) & 1u;
}

__device__ __forceinline__ uint32_t get_base(const uint64_t* w, uint32_t pos) {
  return (uint32_t)(w[pos >> 5] >> (62 - 2 * (pos & 31))) & 3u;
}

// ---- k-mer words -------------------------------------------------------------

// Reverse the order of the 32 two-bit groups of a word.
__device__ __forceinline__ uint64_t rev2(uint64_t x) {
  x = ((x >> 2) & 0x3333333333333333ull) | ((x & 0x3333333333333333ull) << 2);
  x = ((x >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((x & 0x0F0F0F0F0F0F0F0Full) << 4);
  return __builtin_bswap64(x);
}

// Forward k-mer at bit offset `bitpos` of a staged base string, as W words
// (most significant first, value right-aligned in 2k bits).
template <int W>
__device__ __forceinline__ void window_words(const uint64_t* bases,
                                             uint32_t bitpos, uint32_t k,
                                             uint64_t (&f)[W]) {
  const int B = 2 * (int)k;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const int hi = B - 64 * j;  // end (exclusive) of word W-1-j, window-relative
    const int lo = hi - 64;
    if (lo >= 0) f[W - 1 - j] = get_bits(bases, bitpos + (uint32_t)lo, 64);
    else f[W - 1 - j] = get_bits(bases, bitpos, (uint32_t)hi);
  }
}

// Reverse complement of a W-word k-mer value (k odd, so 64W - 2k in 2..62).
template <int W>
__device__ __forceinline__ void revcomp_words(const uint64_t (&f)[W],
                                              uint32_t k, uint64_t (&r)[W]) {
  uint64_t t[W];
#pragma unroll
  for (int j = 0; j < W; ++j) t[j] = rev2(~f[W - 1 - j]);
  const uint32_t s = 64u * W - 2u * k;
#pragma unroll
  for (int j = W - 1; j >= 0; --j)
    r[j] = (t[j] >> s) | (j > 0 ? (t[j - 1] << (64 - s)) : 0ull);
}

// Lexicographic (= numeric) a < b over W words, most significant first.
template <int W>
__device__ __forceinline__ bool words_less(const uint64_t (&a)[W],
                                           const uint64_t (&b)[W]) {
#pragma unroll
  for (int j = 0; j < W; ++j)
    if (a[j] != b[j]) return a[j] < b[j];
  return false;
}

// Owner of a k-mer when the k-mer space is split into `shards` parts (one
// per device in a multi-GPU run): fold the export words, most significant
// first, through the SplitMix64 output function (h = mix(h ^ word), from
// h = 0) and take h mod shards.  The function is part of the interface: a
// caller that splits the work must use the same partition everywhere.
__device__ __forceinline__ uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <int W>
__device__ __forceinline__ uint32_t owner_of(const uint64_t (&key)[W], uint32_t shards) {
  uint64_t h = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) h = splitmix_out(h ^ key[j]);
  return (uint32_t)(h % shards);
}

// Number of 62-bit chunks a k-mer is stored as in the hash table.
__host__ __device__ __forceinline__ int table_chunks(uint32_t k) {
  return (int)((k + 30) / 31);
}

constexpr uint64_t kMask62 = (1ull << 62) - 1;
constexpr uint64_t kOccupied = 1ull << 63;

// Split the 2k-bit value into 62-bit chunks, least significant chunk first
// (c[0] = bits 0..61), and set bit 63 of each, so a stored chunk is never 0
// (0 marks an empty word).  C >= ws; the first `ws` entries of c are written.
template <int W, int C>
__device__ __forceinline__ void to_chunks(const uint64_t (&f)[W], int ws,
                                          uint64_t (&c)[C]) {
#pragma unroll
  for (int cc = 0; cc < C; ++cc) {
    if (cc < ws) {
      const int lo = 62 * cc;
      const int wi = lo >> 6, off = lo & 63;
      uint64_t v = f[W - 1 - wi] >> off;
      if (off > 2 && wi + 1 < W) v |= f[W - 2 - wi] << (64 - off);
      c[cc] = (v & kMask62) | kOccupied;
    }
  }
}

// Inverse of to_chunks: stored chunks (least significant first) -> W export
// words (most significant first).
template <int W>
__device__ __forceinline__ void from_chunks(const uint64_t* c, int ws,
                                            uint64_t (&f)[W]) {
  uint64_t l[W];
#pragma unroll
  for (int j = 0; j < W; ++j) l[j] = 0;
  for (int cc = 0; cc < ws; ++cc) {
    const uint64_t v = c[cc] & kMask62;
    const int lo = 62 * cc;
    const int wi = lo >> 6, off = lo & 63;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      if (j == wi) l[j] |= v << off;
      if (j == wi + 1 && off > 2) l[j] |= v >> (64 - off);
    }
  }
#pragma unroll
  for (int j = 0; j < W; ++j) f[j] = l[W - 1 - j];
}

// MurmurHash3 64-bit finalizer (Appleby): a bijective avalanche mix.
__device__ __forceinline__ uint64_t fmix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

template <int C>
__device__ __forceinline__ uint64_t hash_chunks(const uint64_t (&c)[C], int ws) {
  uint64_t h = 0x9e3779b97f4a7c15ull;
#pragma unroll
  for (int j = 0; j < C; ++j)
    if (j < ws) h = fmix64(h ^ c[j]);
  return h;
}

// ---- hash table slots ----------------------------------------------------
// ws == 1 (k <= 31): 32-byte slot  [chunk0 @0][X @8][SL @16][SR @24]
// ws >= 2          : 64-byte slot  [chunks 0..ws-1 @0..40, least
//                                   significant first][X @40][SL @48][SR @56]
// X  = packed counter, one returning 64-bit add per occurrence: count in bits
//      0-15, left tallies A,C,G,T in 6-bit fields at bits 16-39, right
//      tallies in 6-bit fields at bits 40-63.
// SL, SR = exact 16-bit left/right tallies of "spill" occurrences -- those
//      that found the count already at kSpillAt or more, whose add to X may
//      have carried across fields.  Because X is a sum mod 2^64, subtracting
//      the spill occurrences' increments (known exactly from SL, SR and the
//      count) leaves the first kSpillAt occurrences' increments, whose fields
//      cannot have overflowed: every tally is then recovered exactly.
// Bit 63 of SR marks a heavy k-mer (its count reached kHeavyCount, so the
//      16-bit fields may have wrapped); its count and tallies come from the
//      heavy-hitter recount, and SL then holds its heavy entry index.
struct SlotLayout {
  uint32_t stride, x_off, sl_off, sr_off;
};

__host__ __device__ __forceinline__ SlotLayout slot_layout(int ws) {
  if (ws == 1) return SlotLayout{32u, 8u, 16u, 24u};
  return SlotLayout{64u, 40u, 48u, 56u};
}

constexpr uint32_t kSpillAt = 63;       // 6-bit tallies hold 63
constexpr uint32_t kHeavyCount = 4096;  // spill tallies stay far below 2^15
constexpr uint64_t kCountMask = 0xffffull;
constexpr uint64_t kHeavyBit = 1ull << 63;

__host__ __device__ __forceinline__ uint64_t x_increment(int L, int R) {
  return 1ull + (L >= 0 ? (1ull << (16 + 6 * L)) : 0ull) +
         (R >= 0 ? (1ull << (40 + 6 * R)) : 0ull);
}

// Exact count and tallies of a non-heavy slot from X, SL, SR.
__host__ __device__ __forceinline__ void decode_slot(uint64_t x, uint64_t sl,
                                                     uint64_t sr, uint32_t& count,
                                                     uint32_t (&l)[4],
                                                     uint32_t (&r)[4]) {
  count = (uint32_t)(x & kCountMask);
  const uint64_t ns = count > kSpillAt ? count - kSpillAt : 0;
  uint64_t spill = ns;
  for (int b = 0; b < 4; ++b) {
    const uint64_t a = (sl >> (16 * b)) & 0xffffull;
    const uint64_t c = (sr >> (16 * b)) & (b == 3 ? 0x7fffull : 0xffffull);
    spill += (a << (16 + 6 * b)) + (c << (40 + 6 * b));
    l[b] = (uint32_t)a;
    r[b] = (uint32_t)c;
  }
  const uint64_t first = x - spill;  // the first kSpillAt occurrences, no carries
  for (int b = 0; b < 4; ++b) {
    l[b] += (uint32_t)((first >> (16 + 6 * b)) & 63u);
    r[b] += (uint32_t)((first >> (40 + 6 * b)) & 63u);
  }
}

// Status bits raised by kernels and read back by the host.
enum : uint32_t {
  kStatusProbeLimit = 1u,   // a key found no slot within the probe limit
  kStatusBadOffsets = 2u,   // offsets decrease or exceed the base count
  kStatusHeavy = 4u,        // a kept k-mer reached kHeavyCount occurrences
  kStatusLongTies = 8u,     // a run of equal sort keys (key prefixes) is long
  kStatusStaging = 16u,     // an owner block's staging rows ran out
};

// Counters block (uint64 each) shared by the count pipeline.
enum : int {
  kCtrStatus = 0,
  kCtrWindows = 1,   // valid windows (before any Bloom screening)
  kCtrL1New = 2,     // Bloom level-1 patterns newly completed
  kCtrL2New = 3,     // Bloom level-2 patterns newly completed
  kCtrRows = 4,      // rows kept by classify
  kCtrClaimed = 5,   // table slots claimed
  kCtrHeavy = 6,     // rows that reached kHeavyCount occurrences
  kCtrPassed = 7,    // windows counted into the table (after any Bloom screen)
  kCtrCount = 8
};

// Wave-aggregated append: returns this lane's position among `pred` lanes
// after a single atomic on *ctr by the wave's first active lane.
__device__ __forceinline__ uint64_t wave_append(unsigned long long* ctr,
                                                bool pred) {
  const uint64_t mask = __ballot(pred);
  const uint32_t lane = __lane_id();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t rank = (uint32_t)__popcll(mask & lt);
  uint64_t base = 0;
  const int leader = mask ? (__ffsll((long long)mask) - 1) : 0;
  if (mask && (int)lane == leader)
    base = atomicAdd(ctr, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader);
  return base + rank;
}

// Block-level sum of a per-thread value, added to *ctr by thread 0.
__device__ __forceinline__ void block_add(unsigned long long* ctr, uint64_t v,
                                          uint64_t* lds4) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds4[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t s = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += lds4[i];
    if (s) atomicAdd(ctr, (unsigned long long)s);
  }
}

// ---- tile staging and extension codes (shared by the window kernels) ----

// Copy the planes of positions [O, O + kSpan) into LDS (outside the read
// set: no bases, every position bad).
__device__ __forceinline__ void stage_tile(const uint64_t* g_bases, const uint64_t* g_hq,
                                           const uint64_t* g_bad, const uint64_t* g_st,
                                           int64_t base_words, int64_t plane_words,
                                           int64_t O, uint64_t* s_bases, uint64_t* s_hq,
                                           uint64_t* s_bad, uint64_t* s_st) {
  const int tid = threadIdx.x;
  for (int i = tid; i < kBaseWords; i += kBlock) {
    const int64_t gw = O / 32 + i;
    s_bases[i] = (gw >= 0 && gw < base_words) ? g_bases[gw] : 0ull;
  }
  for (int i = tid; i < kPlaneWords; i += kBlock) {
    const int64_t gw = O / 64 + i;
    const bool in = gw >= 0 && gw < plane_words;
    s_hq[i] = in ? g_hq[gw] : 0ull;
    s_bad[i] = in ? g_bad[gw] : ~0ull;
    s_st[i] = in ? g_st[gw] : 0ull;
  }
}

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

}  // namespace kh
