// Internal interfaces between the host library and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kh_device.hpp"

namespace kh {

struct PackArgs {
  const uint8_t* seq;
  const uint8_t* qual;
  const int64_t* offsets;
  int64_t n_reads;
  int64_t n;            // bases
  int qual_offset, qual_cutoff;
  uint64_t* bases;      // base_words
  uint64_t* hq;         // plane_words each
  uint64_t* bad;
  uint64_t* st;
  int64_t plane_words;
  unsigned long long* ctr;
};

// A k-mer that reached kHeavyCount occurrences (beyond its packed tallies),
// with its exact count and extension tallies (left A,C,G,T then right
// A,C,G,T) from the heavy-hitter recount, and its table slot.
struct HeavyEntry {
  uint64_t chunks[5];
  uint32_t slot, count;
  uint32_t ext[8];
};
static_assert(sizeof(HeavyEntry) == 80, "heavy entry layout");

constexpr uint32_t kHeavyEmpty = 0xffffffffu;
constexpr uint32_t kHeavyMax = 1u << 20;  // heavy k-mers per table

// One tile of a batched launch over several read sets (serving): the tile's
// packed planes, the window starts it covers and the table it updates.
struct TileDesc {
  const uint64_t* bases;
  const uint64_t* hq;
  const uint64_t* bad;
  const uint64_t* st;
  int64_t base_words, plane_words;  // allocated words of the planes
  int64_t p0;                       // first window start (a multiple of 64)
  int64_t hi;                       // end of the chunk (a read boundary):
                                    // windows must satisfy p + k <= hi
  uint8_t* table;
  uint64_t capacity;
  unsigned long long* counters;     // [0] slots claimed, [1] windows counted
  uint64_t* overflow;               // windows that found no slot: entries
  unsigned long long* overflow_n;   //   (descriptor index << 10 | window in tile)
  uint64_t overflow_cap;
  HeavyEntry* heavy;                // heavy recount only
  const uint32_t* heavy_index;
  uint32_t heavy_mask, pad;
};

struct WindowArgs {
  const uint64_t* bases;
  const uint64_t* hq;
  const uint64_t* bad;
  const uint64_t* st;
  int64_t base_words, plane_words, n;
  uint32_t k;
  uint8_t* table;
  uint64_t capacity;
  uint32_t max_probe;
  uint64_t* bloom;       // one word per block: level 1 bits 0-31, level 2 bits 32-63
  uint64_t bloom_blocks;
  // One bit per window start (64 per word, by position): set by pass A when
  // the window was not its key's first sighting, which guarantees the key's
  // level-2 pattern is complete once pass A ends, so pass B counts such a
  // window without loading the filter.  nullptr: pass B loads it for every
  // window.
  uint64_t* seen;
  int count_windows;     // pass B also counts windows (no Bloom pass before it)
  unsigned long long* ctr;
  // heavy-hitter recount (mode 3): exact 32-bit tallies for listed k-mers
  HeavyEntry* heavy;
  const uint32_t* heavy_index;  // open addressing over heavy entries
  uint32_t heavy_mask;          // index size - 1 (power of two)
  // batched launch: one descriptor per block (nullptr: the fields above)
  const TileDesc* tiles;
  int64_t n_tiles;
  // launch shape (0 = default): windows per lane in a sub-pass (1, 2, 4) and
  // tiles per block (one read set only)
  int lanes;
  int tiles_per_block;
  // keep only the keys of part `owner` of `shards` (0 or 1: every key)
  uint32_t shards, owner;
  // counting pass (mode 2, one read set, no key-space parts): merge each
  // tile's repeated k-mers in LDS first (k_count_agg); blocks then take
  // consecutive tiles
  int aggregate;
  // one read set, modes 0, 1 and 3: tiles [t_begin, t_end) (t_end 0: to the
  // last), for passes that run while later reads are still being uploaded
  int64_t t_begin, t_end;
};

// Bloom pass A for several k of one key width over one packed read set (one
// launch).  Per-k parameters live in device memory so the kernel reads them
// with uniform (scalar) loads.
struct BloomSlot {
  uint32_t k, pad;
  uint64_t* bloom;
  uint64_t bloom_blocks;
  unsigned long long* ctr;  // counters of this k
  uint64_t* seen;           // this k's sighting bits (WindowArgs::seen)
};

constexpr int kBloomFuse = 3;  // k per fused Bloom launch

struct MultiBloomArgs {
  const uint64_t* bases;
  const uint64_t* hq;
  const uint64_t* bad;
  const uint64_t* st;
  int64_t base_words, plane_words, n;
  int nk;                    // 1..kBloomFuse
  uint32_t k0;               // any k of the launch (they share one key width)
  const BloomSlot* slots;    // nk entries, device memory
  int lanes;                 // launch shape, as in WindowArgs
  int tiles_per_block;
  uint32_t shards, owner;    // key-space part, as in WindowArgs
  int64_t t_begin, t_end;    // tiles [t_begin, t_end) (t_end 0: to the last)
};

struct ClassifyArgs {
  const uint8_t* table;
  uint64_t capacity;
  uint32_t k, min_count;
  uint64_t* pfx_out;     // capacity: sort key of each kept row (whole key for
                         // k <= 31, else its top kSortPrefixBits bits)
  uint32_t* idx_out;     // capacity: its slot
  uint32_t* heavy_list;  // kHeavyMax slot indices of heavy k-mers
  unsigned long long* ctr;
};

struct HeavyBuildArgs {
  uint8_t* table;
  uint32_t k;
  const uint32_t* heavy_list;
  uint32_t n_heavy;
  HeavyEntry* heavy;
  uint32_t* heavy_index;
  uint32_t heavy_mask;
};

struct GatherArgs {
  const uint8_t* table;
  const HeavyEntry* heavy;  // exact count and tallies of heavy rows
  uint64_t* keys;           // n_rows * W export words
  const uint32_t* idx;
  int64_t n_rows;
  uint32_t k, t_min_ext, t_base, err_ppm;
  uint32_t* counts;
  uint32_t* ext;
  uint8_t* codes;
};

// ---- owner-partitioned counting (kh_owner.hip) ----
constexpr int kOwnL1Max = 1024;       // level-1 buckets at most (p1 <= 10)
constexpr int kOwnRouteThreads = 1024;  // level-1 block: one window per lane per tile
constexpr int kOwnL2Max = 11;         // level-2 digit bits at most
constexpr int kOwnPartThreads = 1024;  // level-2 partition block
constexpr int kOwnThreads = 1024;      // owner block
constexpr int kOwnBlocksPerCU = 1024 / kOwnThreads;  // owner blocks sharing a CU's LDS
constexpr int kOwnLdsBytes = 160 * 1024 / kOwnBlocksPerCU;  // LDS of one owner block
constexpr int kOwnBloomBits = kOwnThreads == 1024 ? 11 : 10;
constexpr int kOwnBloomWords = 1 << kOwnBloomBits;  // owner Bloom filter (8 B words)
constexpr int kOwnSortBits = kOwnBloomBits - 1;     // owner sort: buckets of the next key bits
constexpr int kOwnStripes = 256;       // copies of the owner counters (contention)
constexpr int kOwnCopyThreads = 256;   // row copy (and key-order sort) block

// Level-1 digit: the top own_p1(k) key bits (1,024 buckets for k >= 5).  A
// record holds only the key bits below it (own_rest_bits), which its bucket
// implies: own_record_words words of (rest << 6 | extension byte), and the
// owners' LDS tables own_chunks 62-bit chunks of the rest.
__host__ __device__ inline int own_p1(uint32_t k) { return 2 * (int)k < 10 ? 2 * (int)k : 10; }
__host__ __device__ inline int own_rest_bits(uint32_t k) { return 2 * (int)k - own_p1(k); }
__host__ __device__ inline int own_record_words(uint32_t k) {
  return (own_rest_bits(k) + 6 + 63) / 64;
}
__host__ __device__ inline int own_chunks(uint32_t k) {
  const int b = own_rest_bits(k);
  return b <= 62 ? 1 : (b + 61) / 62;
}

// Routing of windows to level-1 buckets (histogram, then emit).
struct OwnRouteArgs {
  const uint64_t* bases;
  const uint64_t* hq;
  const uint64_t* bad;
  const uint64_t* st;
  int64_t base_words, plane_words, n;
  uint32_t k, shards, owner, p1;
  uint32_t* h1;             // (1 << p1) x grid matrix, bucket-major
  uint64_t* rec;            // emit: records, R words each
  unsigned long long* ctr;  // kCtrWindows
};

// A level-1 bucket: its records [start, start + n), split by its next p2
// key bits into 2^p2 owners (ids sbbase ...), read in `chunks` chunks (ids
// cbase ...), whose digit counts are the chunk-major matrix entries
// m[mbase + chunk * 2^p2 + digit].
struct OwnBucket {
  uint64_t start, n, mbase;
  uint32_t p2, chunks, sbbase, cbase;
};

struct OwnPartArgs {
  const uint64_t* rec_in;
  uint64_t* rec_out;
  const OwnBucket* buckets;
  int n_buckets;
  uint32_t* m;
  uint32_t* start2;  // n_owners + 1: record counts, then (scanned) first records
  uint16_t* owner_bucket;  // bucket of each owner (k_own_maps)
  uint8_t* owner_pfx;      // key bits an owner's keys share (p1 + its bucket's p2)
  uint16_t* chunk_bucket;  // bucket of each level-2 chunk
  uint32_t k, p1;
};

struct OwnCountArgs {
  const uint64_t* rec;
  const uint32_t* start2;
  const uint16_t* owner_bucket;  // level-1 bucket (top key bits) of each owner
  uint32_t n_owners;
  uint32_t k, p1, min_count, t_min_ext, t_base, err_ppm, use_bloom;
  uint32_t slots;          // table slots used (<= own_slots(k); a testing hook)
  uint64_t* st_keys;       // st_cap staging rows
  uint32_t* st_counts;
  uint32_t* st_ext;
  uint8_t* st_codes;
  uint64_t st_cap;
  uint64_t st_chunk;       // staging rows a block takes from the cursor at a time
  unsigned long long* st_cursor;  // next untaken staging row (zero at launch)
  const uint32_t* st_fixed;  // nullptr, or every owner's first staging row
  uint64_t* st_off;        // first staging row of each owner
  uint32_t* rows_sb;       // rows of each owner
  uint32_t* row_off;       // rows of each owner (scanned into offsets later)
  unsigned long long* ctr;  // kOwnStripes x kCtrCount counters (summed by the host)
  unsigned long long* prof; // 8 phase clocks or nullptr
};

struct OwnCopyArgs {
  const uint8_t* owner_pfx;  // key bits each owner's keys share
  uint32_t k;
  const uint64_t* st_keys;
  const uint32_t* st_counts;
  const uint32_t* st_ext;
  const uint8_t* st_codes;
  const uint32_t* rows_sb;
  const uint32_t* row_off;
  const uint64_t* st_off;  // first staging row of each owner
  uint32_t W;
  uint64_t* keys;
  uint32_t* counts;
  uint32_t* ext;
  uint8_t* codes;
};

int own_chunk_records(uint32_t k);
int own_slots(uint32_t k);
void launch_own_hist(const OwnRouteArgs& a, int grid, hipStream_t s);
void launch_own_emit(const OwnRouteArgs& a, int grid, hipStream_t s);
void launch_own_part(const OwnPartArgs& a, uint32_t n_chunks, int scatter, hipStream_t s);
void launch_own_maps(const OwnPartArgs& a, hipStream_t s);
void launch_own_colscan(const OwnPartArgs& a, uint32_t n_owners, hipStream_t s);
// blocks: persistent blocks (at most one per owner), one per compute unit
void launch_own_count(const OwnCountArgs& a, uint32_t blocks, hipStream_t s);
void launch_own_copy(const OwnCopyArgs& a, uint32_t n_owners, hipStream_t s);
void launch_gather_strided(const uint32_t* src, uint64_t stride, uint32_t n, uint32_t* dst,
                           hipStream_t s);

void launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);
void launch_reset_ctr(unsigned long long* ctr, uint64_t keep, hipStream_t s);
void launch_pack(const PackArgs& a, hipStream_t s);
// The two halves of launch_pack: bases, quality and non-base planes of the
// positions [p0, p1) (p0 a multiple of 64; p1 a multiple of 64 or n), and
// the read-start plane with the offsets check.
void launch_pack_range(const PackArgs& a, int64_t p0, int64_t p1, hipStream_t s);
void launch_mark_starts(const PackArgs& a, hipStream_t s);
void launch_windows(const WindowArgs& a, int mode, hipStream_t s);
void launch_bloom_multi(const MultiBloomArgs& a, hipStream_t s);

// Count the windows listed in an overflow list (see TileDesc) into the tables
// their descriptors now name (grown so that every listed window finds a
// slot); claimed slots are added to each descriptor's counters[0].
void launch_replay(const TileDesc* descs, const uint64_t* entries, uint64_t n,
                   uint32_t k, hipStream_t s);

// Move every occupied slot of `old_table` into `new_table` (zeroed, larger).
void launch_rehash(const uint8_t* old_table, uint64_t old_cap, uint8_t* new_table,
                   uint64_t new_cap, uint32_t k, unsigned long long* ctr,
                   hipStream_t s);
void launch_classify(const ClassifyArgs& a, hipStream_t s);
void launch_gather(const GatherArgs& a, hipStream_t s);
void launch_heavy_build(const HeavyBuildArgs& a, hipStream_t s);

// The sort key of a row: its whole key for k <= 31, else the top
// kSortPrefixBits bits (20 bases; keys rarely share them, and each pass of
// the radix sort costs as much as the table scan).  Rows sorted by prefix:
// order every run of equal prefixes by the full key (read from the table
// through the slot index).  Runs longer than kMaxTieRun are left alone and
// raise kStatusLongTies.
constexpr int kSortPrefixBits = 40;
constexpr int kMaxTieRun = 64;
void launch_fix_ties(const uint64_t* pfx, uint32_t* idx, int64_t n,
                     const uint8_t* table, uint32_t k, unsigned long long* ctr,
                     hipStream_t s);
// Full export keys of rows (through the slot index), for the full-key sort.
void launch_row_keys(const uint32_t* idx, int64_t n, const uint8_t* table,
                     uint32_t k, uint64_t* keys, hipStream_t s);

// LSD radix sort of n rows of W key words (row-major, most significant word
// first) with a uint32 payload, ascending by key; `bits0` = significant bits
// of word 0.  Buffers a/b are ping-pong storage of n rows each; the result
// lands in the returned set (0 = a, 1 = b).  tmp must hold sort_tmp_words(n)
// uint32 values.
uint64_t sort_tmp_words(int64_t n);
// In-place exclusive scan of m 32-bit values; part must hold
// scan_tmp_words(m) words.
uint64_t scan_tmp_words(int64_t m);
void exclusive_scan_u32(uint32_t* x, int64_t m, uint32_t* part, hipStream_t s);

// Sort n rows of one-word keys of `bits` significant bits (with their uint32
// payload) ascending; rows with equal keys end in any order.  Up to 16,384
// rows are sorted in LDS by one launch; larger sets take the segmented sort
// (top bits by LSD passes, then segments of buckets sorted in LDS), which
// needs seg_sort_bytes(n, bits) bytes of device scratch (0: the plain LSD
// sort is used, scratch may be null) and synchronises the stream.  The
// result lands in set *which (0 = a, 1 = b).  Returns 0, or 1 if a HIP call
// failed.
uint64_t seg_sort_bytes(int64_t n, int bits);
int sort_rows(uint64_t* keys_a, uint32_t* idx_a, uint64_t* keys_b, uint32_t* idx_b,
              int64_t n, int bits, uint32_t* tmp, void* scratch, hipStream_t s, int* which);
int radix_sort(uint64_t* keys_a, uint32_t* idx_a, uint64_t* keys_b,
               uint32_t* idx_b, int64_t n, int W, int bits0, uint32_t* tmp,
               hipStream_t s);

}  // namespace kh
