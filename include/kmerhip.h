/*
 * kmerhip -- k-mer analysis on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library.  Reads with qualities go in; k, the count threshold
 * and the quality cutoff are parameters; a table of canonical k-mers with
 * their counts, extension tallies and two-letter extension codes comes out.
 * This is the "K-mer Analysis" stage of the paper (Section II-B): split reads
 * into k-mers overlapping by k-1 bases, count them, keep those seen often
 * enough, and record each k-mer's extensions; Section II-C gives the output
 * form (key plus a code [ACGT][ACGT] naming the unique preceding/following
 * bases) and the depth-adaptive rule deciding whether an extension is unique.
 *
 * Conventions used by every call
 *   - Bases are A, C, G, T (either case).  Any other byte (N, IUPAC, ...) is
 *     not a base: a window that holds one is not a k-mer, and such a
 *     neighbour is not an extension.
 *   - Canonical k-mer: the lexicographically smaller of a k-mer and its
 *     reverse complement (A < C < G < T).  k must be odd, so no k-mer is its
 *     own reverse complement.  When the reverse complement is the key, the
 *     left and right neighbours swap sides and are complemented.
 *   - Key value: N = sum_j code(s_j) * 4^(k-1-j) with A=0, C=1, G=2, T=3.
 *     A key is W = ceil(k/32) uint64 words, most significant word first, so
 *     comparing words in order compares k-mers lexicographically.
 *   - A neighbour base counts as an extension observation only when its
 *     Phred score (quality byte - qual_offset) is >= qual_cutoff.  The
 *     qualities of the k-mer's own bases never matter.
 *   - Every row has count >= min_count.  Rows are sorted ascending by key.
 *   - Extension code per side, from the tallies c[A..T] of that side and the
 *     k-mer's count d:  m = max c; 'X' (dead end) if m < t_min_ext;
 *     'F' (fork) if two or more bases tie at m; otherwise, with
 *     alt = sum c - m, the base letter if alt * 10^6 <= max(t_base * 10^6,
 *     err_ppm * d) (no more than t_hq = max(t_base, e * d) contradicting
 *     observations, e = err_ppm / 10^6), else 'F'.
 *
 * Errors.  Every call returns KH_OK (0) or a positive KH_E* code; no C++
 * exception crosses this boundary.  kh_last_error() returns a message for
 * the calling thread's most recent failure.
 *
 * Streams.  Calls that take `stream` (a hipStream_t, NULL = the null stream)
 * enqueue their device work on it.  kh_count and kh_count_multi_k return
 * after the result's row count is known (they synchronise the stream at
 * planning points); the rows themselves are valid once the stream reaches
 * the end of the call's work, which is already the case on return.
 *
 * Thread safety.  One kh_ctx must not be used by two threads at once.
 * Different contexts are independent.
 */
#ifndef KMERHIP_H
#define KMERHIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KH_OK = 0,
  KH_EINVAL = 1,    /* bad argument: NULL pointer, even or out-of-range k,
                       min_count 0, offsets not starting at 0 or decreasing */
  KH_ENOMEM = 2,    /* the plan exceeds the context's HBM budget, or a device
                       allocation failed */
  KH_EOVERFLOW = 3, /* a counter would exceed its width: more than 2^32-1
                       windows in one table, or more than 2^20 distinct
                       k-mers with 4096 or more occurrences */
  KH_EAGAIN = 4,    /* serving: the request cannot be admitted now */
  KH_EDEVICE = 5,   /* a HIP runtime call failed, or no usable gfx950 device */
  KH_ENOTFOUND = 6  /* serving: unknown sample or ticket */
};

typedef struct kh_ctx kh_ctx;
typedef struct kh_table kh_table;

/* A read set: read r is seq[offsets[r] .. offsets[r+1]) with the quality
 * bytes qual[same range].  offsets has n_reads + 1 non-decreasing entries and
 * offsets[0] == 0; the total base count is offsets[n_reads].  Mates of a pair
 * are two independent reads (no k-mer spans the insert).  With on_device = 0
 * the three arrays are host memory and are copied to the device; with 1 they
 * are device memory of the context's GPU.  The caller owns the buffers and
 * may reuse them once the call returns. */
typedef struct {
  const char *seq;
  const char *qual;
  const int64_t *offsets;
  int64_t n_reads;
  int32_t on_device;
} kh_reads;

/* Parameters.  kh_default_params fills the documented defaults. */
typedef struct {
  uint32_t k;           /* k-mer length, odd, 1..127 */
  uint32_t min_count;   /* keep k-mers with count >= min_count, 1..4096; 2
                           drops singletons ("more than eps times" is
                           eps + 1) */
  uint32_t qual_offset; /* Phred encoding offset, default 33 */
  uint32_t qual_cutoff; /* extension quality cutoff, default 20 */
  uint32_t t_min_ext;   /* dead-end threshold, default 2 */
  uint32_t t_base;      /* floor of the contradiction threshold, default 1 */
  uint32_t err_ppm;     /* error-model slope e in parts per million,
                           default 5000 (e = 0.005) */
  uint32_t use_bloom;   /* 1: two-pass Bloom filter screens out k-mers seen
                           once before they reach the table (needs
                           min_count >= 2); the result is identical */
  uint32_t bloom_bits;  /* Bloom bits per level per base position (<= 64),
                           0 = the context's tuning (default 2) */
  float load_factor;    /* target table load in [0, 0.95), 0 = the
                           context's tuning (default 0.5) */
  uint32_t owner_shards; /* k-mer space split into this many parts (one per
                            device of a multi-GPU run; 0 or 1 = no split): the
                            call counts only the k-mers of part `owner`
                            (kh_owner_of), and n_windows counts only their
                            windows.  Not for serving. */
  uint32_t owner;        /* < owner_shards */
} kh_params;

void kh_default_params(kh_params *p, uint32_t k);

/* Part of the k-mer space that owns a canonical key of W words (most
 * significant first, as exported): h = 0, then h = mix(h ^ word) for each
 * word in order, where mix is the SplitMix64 output function
 * (z ^= z >> 30; z *= 0xbf58476d1ce4e5b9; z ^= z >> 27;
 * z *= 0x94d049bb133111eb; z ^= z >> 31); the owner is h mod shards.
 * Returns 0 for shards <= 1 or a NULL key. */
uint32_t kh_owner_of(const uint64_t *key, uint32_t W, uint32_t shards);

/* Device memory from the caller, e.g. a framework's caching allocator:
 * alloc returns `bytes` of memory of HIP device `device` (NULL when it has
 * none), free takes back a block alloc returned, with the same size.  The
 * library calls them under the context's lock (never two at once for one
 * context), possibly from its own threads (a server's worker).  Blocks are
 * freed at kh_trim and kh_destroy, and when a request would pass the budget
 * or alloc fails, always after the device has finished the work using them
 * (the library synchronizes the device first). */
typedef void *(*kh_alloc_fn)(uint64_t bytes, int device, void *user);
typedef void (*kh_free_fn)(void *ptr, uint64_t bytes, int device, void *user);

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the context holds at any time (0 = no cap beyond the device).
 * Device memory is drawn from a caching pool owned by the context and reused
 * across calls; the pool takes its blocks from alloc_fn / free_fn (with
 * `user`) when both are given, else from hipMalloc / hipFree (then blocks of
 * a destroyed context are kept for the next context on the device).
 * KH_EINVAL if only one of alloc_fn and free_fn is given. */
int kh_create(kh_ctx **out, int device, uint64_t hbm_budget_bytes,
              kh_alloc_fn alloc_fn, kh_free_fn free_fn, void *user);

/* Destroy a context.  Its device memory goes back to free_fn, or, from
 * hipMalloc, to a cache kept per device for the next context created there
 * (see kh_release_cached).  Tables created
 * from it that are still alive lose their rows (n_rows becomes 0); they must
 * still be released with kh_table_free. */
int kh_destroy(kh_ctx *ctx);

/* Return the blocks the context's pool keeps for reuse to the driver (tables
 * and contigs alive keep theirs). */
int kh_trim(kh_ctx *ctx);

/* Return the device memory kept from destroyed contexts on `device` to the
 * driver.  Contexts and servers alive on the device keep theirs.  Not to be
 * called while a context is being created or destroyed on that device.
 * KH_EINVAL for a device out of range, KH_EDEVICE without a device. */
int kh_release_cached(int device);

/* Message of the calling thread's most recent failure ("" if none). */
const char *kh_last_error(void);

/* Count the k-mers of one read set (one k).  On success *out is a table
 * owned by the library until kh_table_free.  Host reads (on_device = 0)
 * with use_bloom are copied in chunks on the context's side stream, the
 * Bloom pass over each chunk overlapping the next chunk's copy.  Errors:
 * KH_EINVAL, KH_ENOMEM, KH_EOVERFLOW, KH_EDEVICE. */
int kh_count(kh_ctx *ctx, const kh_reads *reads, const kh_params *params,
             void *stream, kh_table **out);

/* Count the same read set at nk values of k in one batched run: the reads
 * are packed once, and each pass handles every k from the same staged tile
 * of bases (the iterative k loop of Algorithm 1 runs k-mer analysis once per
 * k on the same reads).  outs[i] is bit-identical to kh_count with
 * k = ks[i] and the other fields of params.  nk <= 8.  Host reads
 * (on_device = 0) with use_bloom are copied in chunks on the context's side
 * stream, each chunk's Bloom pass overlapping the next chunk's copy; the
 * host buffers are read until the call returns. */
int kh_count_multi_k(kh_ctx *ctx, const kh_reads *reads,
                     const kh_params *params, const uint32_t *ks, int nk,
                     void *stream, kh_table **outs);

/* Shape of a table: k, W = ceil(k/32), number of rows, and the number of
 * valid windows counted before the threshold (the sum of all counts). */
int kh_table_info(const kh_table *t, uint32_t *k, uint32_t *W,
                  int64_t *n_rows, uint64_t *n_windows);

/* Copy the rows out.  Any destination may be NULL to skip it.  Layout:
 * keys n_rows*W uint64 (row-major), counts n_rows uint32, ext n_rows*8
 * uint32 (left A,C,G,T then right A,C,G,T), codes n_rows*2 bytes (left,
 * right letters in {A,C,G,T,F,X}).  dst_on_device selects device or host
 * destinations; the caller allocates them.  Synchronous with respect to
 * `stream`. */
int kh_table_export(const kh_table *t, uint64_t *keys, uint32_t *counts,
                    uint32_t *ext, uint8_t *codes, int dst_on_device,
                    void *stream);

/* Device pointers of the rows (valid until kh_table_free).  Any output may
 * be NULL. */
int kh_table_device_rows(const kh_table *t, const uint64_t **keys,
                         const uint32_t **counts, const uint32_t **ext,
                         const uint8_t **codes);

/* Release a table (its device rows return to the context's pool).  NULL is
 * accepted. */
int kh_table_free(kh_table *t);

/* Heavy hitters (Section II-B: k-mers occurring so often, e.g. in highly
 * abundant organisms, that they need dedicated treatment; every count here
 * is exact, k-mers reaching 4096 occurrences being recounted by a separate
 * pass): the rows of t whose count is >= min_count (>= 1), in key order.
 * Up to cap rows go to host buffers keys_out (W words per row) and
 * counts_out; *n_out receives the number of such rows (it may exceed cap:
 * call again with larger buffers).  Synchronous with respect to stream. */
int kh_heavy_hitters(const kh_table *t, uint32_t min_count, void *stream,
                     uint64_t *keys_out, uint32_t *counts_out, int64_t cap,
                     int64_t *n_out);

/* Timing of the device phases of the context's most recent kh_count /
 * kh_count_multi_k call, in milliseconds (HIP events on the call's stream):
 * [0] pack, [1] Bloom pass, [2] count pass, [3] classify + compact,
 * [4] sort, [5] gather.  With the owner-partitioned count (kh_tuning
 * partitioned = 1): [1] routing of the windows to their owners (both
 * partition passes), [2] the owner pass (Bloom screen, count and classify
 * in LDS), [3] 0, [4] the row-offset scan, [5] the copy of the owners' rows
 * into the table, sorted by key within each owner.  Filled only when timing
 * is enabled. */
int kh_set_timing(kh_ctx *ctx, int enable);
int kh_last_timing(const kh_ctx *ctx, float ms[6]);

/* Statistics of the context's most recent count (the last k of a multi-k
 * call): [0] table capacity (slots), [1] slots claimed, [2] Bloom level-1
 * patterns completed, [3] Bloom level-2 patterns completed, [4] valid
 * windows, [5] rows kept, [6] table rebuilds after a probe ran out, [7] table
 * bytes, [8] windows counted into the table (after the Bloom screen),
 * [9] heavy k-mers recounted, [10] k, [11] 1 if rows needed the full-key
 * sort (many keys sharing their top 20 bases), else 0.  With the
 * owner-partitioned count: [0] owners x LDS slots, [1] keys the owners
 * inserted, [6] finer re-splits after an owner's keys did not fit, [7] bytes
 * of the routed records and the owners' staging rows, [9] owners whose keys
 * did not fit their table (over every split tried), [11] keys of the
 * fullest owner (counts are exact 32-bit LDS counters: no heavy recount). */
int kh_last_stats(const kh_ctx *ctx, uint64_t out[12]);

/* *graphed = 1 if the context's most recent batched kh_count_multi_k call
 * (two or more k) ran its counting passes as one replayed HIP graph, 0 if it
 * launched them one by one (graph capture unavailable). */
int kh_last_graphed(const kh_ctx *ctx, int *graphed);

/* Phase times (as kh_last_timing) and statistics (as kh_last_stats) of the
 * i-th k of the context's most recent kh_count / kh_count_multi_k call
 * (i < 8).  The shared pack phase is booked on i = 0. */
int kh_last_k_report(const kh_ctx *ctx, int i, float ms[6], uint64_t stats[12]);

/* ---- Contigs (de Bruijn graph traversal) ---------------------------------
 * Section II-C: the kept k-mers of a table are the vertices of the de Bruijn
 * graph, their two-letter codes its edges; a contig is a maximal path of
 * k-mers joined by unique high-quality extensions.  Precisely: k-mer S
 * joins S' = S[1..k) + b when S's right code is b, S' is a row of the table
 * and S''s left code is S[0] (codes of a k-mer read on its reverse strand
 * swap sides and complement); an edge from a k-mer to itself or to its own
 * reverse complement is dropped.  Every row is in exactly one contig: a
 * maximal path, written in the orientation that is lexicographically
 * smaller than its reverse complement, or a cycle, opened at its smallest
 * k-mer in canonical orientation and written walking right (n k-mers give
 * k + n - 1 bases).  Contigs are listed by their smallest k-mer. */
typedef struct kh_contigs kh_contigs;

/* Contigs of table t (rows on the device of ctx).  Stream-ordered on
 * hip_stream; returns after the contigs are complete.  *out is freed with
 * kh_contigs_free.  Besides the sequences the contigs keep the contig of
 * every row of t (4 bytes per row), which kh_prune and kh_localize_reads
 * use.  KH_EINVAL for a table of a destroyed context or another device,
 * KH_ENOMEM if the working set (about 70 bytes per row) does not fit. */
int kh_traverse(kh_ctx *ctx, const kh_table *t, void *hip_stream,
                kh_contigs **out);

/* Sizes: k, number of contigs, bases over all contigs, k-mers lying on
 * cycles, pointer-jumping rounds run.  Any pointer may be NULL. */
int kh_contigs_info(const kh_contigs *c, uint32_t *k, int64_t *n_contigs,
                    int64_t *total_bases, int64_t *cycle_kmers, int *rounds);

/* Copy out (caller allocates; NULL skips a field): seq total_bases ASCII
 * bytes (contigs back to back, no separators), offsets n_contigs + 1,
 * n_kmers n_contigs, depth n_contigs (sum of the k-mers' counts), cycle
 * n_contigs (1 for a cycle).  dst_on_device selects device destinations. */
int kh_contigs_export(const kh_contigs *c, char *seq, int64_t *offsets,
                      int64_t *n_kmers, uint64_t *depth, uint8_t *cycle,
                      int dst_on_device);

/* Device pointers to the contigs' sequence and offsets (valid until
 * kh_contigs_free), e.g. to merge them into the next k's table. */
int kh_contigs_device(const kh_contigs *c, const char **seq,
                      const int64_t **offsets);

/* Release contigs (NULL accepted).  Contigs of a destroyed context keep no
 * data (n_contigs becomes 0) and must still be freed. */
int kh_contigs_free(kh_contigs *c);

/* Algorithm 1's Merge (Section II, merging k-mer sets): the k-mers of
 * contigs assembled with a smaller k join table t as error-free k-mers with
 * unique high-quality extensions.  A k-mer that is a row of t keeps its row;
 * a new one becomes a row with count 0, no tallies, and per side the code:
 * the neighbouring contig base when every occurrence has one and they agree,
 * 'X' when none has one, 'F' otherwise.  Contig windows holding a byte other
 * than A/C/G/T (either case) are skipped.  seq holds the contigs back to
 * back (ASCII), offsets n_contigs + 1 entries; both on the device if
 * on_device.  *out (t's k, rows in key order, n_windows of t) is freed with
 * kh_table_free; t is unchanged. */
int kh_merge_contigs(kh_ctx *ctx, const kh_table *t, const char *seq,
                     const int64_t *offsets, int64_t n_contigs, int on_device,
                     void *hip_stream, kh_table **out);

/* ---- Iterative graph pruning (Algorithm 2) ---------------------------------
 * Section II, iterative graph pruning (after IDBA-UD): a depth threshold tau
 * starts at 1 and grows by the factor (1 + alpha) after every sweep while it
 * is below the largest depth of the contigs left; each sweep removes every
 * contig of at most 2k bases whose depth is at most
 * min(tau, beta * neighbourhood depth).  Precisely: depth = the mean count
 * of the contig's k-mers; the neighbours of c are the other contigs holding
 * a k-mer that overlaps c's first k-mer by k-1 bases on its left or its last
 * k-mer by k-1 bases on its right (any base, either strand), each counted
 * once; the neighbourhood depth pools the neighbours still present (sum of
 * their counts / number of their k-mers); a contig with no neighbour left
 * stays; a sweep decides on the contigs as they were when it started.
 * Arithmetic is IEEE double, one rounding per operation: d = sum / n,
 * nd = sum / n, remove iff d <= min(tau, beta * nd); tau = tau * (1 + alpha)
 * with 1 + alpha rounded once.  The paper gives no values for alpha and
 * beta. */
typedef struct {
  double alpha; /* tau grows by the factor 1 + alpha per sweep, in
                   [0.001, 1000]; default 0.1 */
  double beta;  /* relative depth cut, in [0, 1e6]; default 0.2 */
} kh_prune_params;

typedef struct {
  int64_t sweeps;   /* sweeps run */
  int64_t removed;  /* contigs removed */
  double tau;       /* the threshold that ended the loop */
  double max_depth; /* largest depth of the contigs left */
} kh_prune_report;

void kh_default_prune_params(kh_prune_params *p);

/* Prune contigs c, which kh_traverse walked from table t (t must still be
 * live: its sorted rows and the traversal's row -> contig map give the
 * neighbours).  params NULL takes the defaults.  *out holds the kept
 * contigs in their order (kh_contigs_free; it cannot be pruned again).
 * removed_at (host, c's n_contigs entries, or NULL) receives for every
 * contig the sweep that removed it, or -1; report (or NULL) the totals.
 * Stream-ordered on hip_stream; returns when done.  KH_EINVAL for
 * parameters out of range, contigs not walked from t, or objects of
 * another device; KH_ENOMEM if the working set (about 80 bytes per contig,
 * plus the kept contigs) does not fit. */
int kh_prune(kh_ctx *ctx, const kh_table *t, const kh_contigs *c,
             const kh_prune_params *params, void *hip_stream, kh_contigs **out,
             int32_t *removed_at, kh_prune_report *report);

/* ---- Read localisation --------------------------------------------------
 * Section II, read localisation: once an iteration has produced contigs,
 * reads of the same contig are brought together so that later iterations
 * find every occurrence of a k-mer within a short stretch of the read
 * stream (the counting table's updates then hit in the caches).  A read's
 * anchor is the first of its windows, in read order, that holds k bases of
 * A/C/G/T (either case) and whose canonical k-mer is a row of t; reads are
 * ordered by the index of the contig holding that row, stably, reads
 * without an anchor last.  Counting does not depend on read order (Section
 * II-A, Use case 1): tables of the permuted reads equal the input's. */

/* Order of the reads grouped by contig: order (n_reads entries, device
 * memory if order_on_device, else host) receives read indices.  c must
 * have been walked from t by kh_traverse (t still live); reads on the host
 * or the device (qualities are not read).  KH_EINVAL for contigs not walked
 * from t, objects of another device, bad offsets or more than 2^32 - 1
 * reads; KH_ENOMEM if the working set (about 28 bytes per read) does not
 * fit. */
int kh_localize_reads(kh_ctx *ctx, const kh_table *t, const kh_contigs *c,
                      const kh_reads *reads, void *hip_stream, int64_t *order,
                      int order_on_device);

/* Reads (device memory) copied in the given order (device, n_reads read
 * indices) into caller-allocated device buffers: seq_out and qual_out of
 * offsets[n_reads] bytes, offsets_out of n_reads + 1 entries.
 * KH_EINVAL if order holds an index out of range or is not a permutation
 * (its reads' lengths do not add up to the input's bases), or for bad
 * offsets; nothing is written to seq_out / qual_out then. */
int kh_gather_reads(kh_ctx *ctx, const kh_reads *reads, const int64_t *order,
                    void *hip_stream, char *seq_out, char *qual_out,
                    int64_t *offsets_out);

/* ---- Tuning ---------------------------------------------------------------
 * Free parameters of the implementation (none changes a result; tables are
 * bit-identical under every setting).  A context starts from
 * kh_default_tuning; kh_params.load_factor and kh_params.bloom_bits left at 0
 * take the context's values. */
typedef struct {
  float load_factor;         /* table load the capacity is planned for, in
                                [0.05, 0.95); default 0.5 */
  uint32_t bloom_bits;       /* Bloom bits per level per base position,
                                1..64; default 2 */
  uint32_t bloom_lanes;      /* windows each lane carries through the Bloom
                                pass at once: 1, 2 or 4; default 4 */
  uint32_t count_lanes;      /* the same for the counting pass: 1, 2 or 4,
                                or 0 = by key width (2 for k = 33..96,
                                else 1); default 2 */
  uint32_t tiles_per_block;  /* 1,024-window tiles each block of a window pass
                                takes in turn, 1..1024 (fewer while a pass
                                would have under 1,024 blocks); default 8 */
  uint32_t aggregate;        /* 1: the reads are first put in the order of
                                their minimizers and the counting pass merges
                                each tile's repeated k-mers in LDS before
                                updating the table (one update per distinct
                                k-mer and tile; k <= 95 with the Bloom screen
                                and without key-space parts, else the plain
                                pass); 0 or 1, default 0 */
  uint32_t tails_overlap;    /* batched call: 1 = each k's classify, sort and
                                gather start when its counting pass ends,
                                beside the later passes; 0 = they start once
                                every counting pass has ended; default 1 */
  uint32_t partitioned;      /* 1: kh_count and kh_count_multi_k route each
                                window to the owner of its key prefix (two
                                streaming partition passes), every owner
                                workgroup runs the Bloom screen, the count
                                and classify in LDS (Section II-B's
                                owner-computes layout), and the copy into
                                the table sorts each owner's rows; k after
                                k, no device hash table.  0: one open-addressing table in
                                HBM per k (the fields above).  A k whose
                                owners' keys do not fit their LDS tables
                                even after two finer splits, or whose two
                                record buffers (16 x ceil((2k - min(10, 2k)
                                + 6) / 64) bytes per window) the HBM budget
                                refuses,
                                is counted with 0.  Not used by
                                kh_count_noalloc, with aggregate = 1, or by
                                serving.  0 or 1, default 1 */
} kh_tuning;

void kh_default_tuning(kh_tuning *t);
int kh_get_tuning(const kh_ctx *ctx, kh_tuning *out);
/* KH_EINVAL for a value out of range (the context keeps its tuning). */
int kh_set_tuning(kh_ctx *ctx, const kh_tuning *t);

typedef struct {
  uint32_t trials;     /* calls timed */
  uint32_t skipped;    /* settings that did not fit in device memory */
  double start_ms;     /* the call under the tuning in force on entry */
  double best_ms;      /* the call under the tuning chosen */
} kh_tune_report;

/* Autotuner: time kh_count_multi_k(reads, params, ks) (params.load_factor
 * and params.bloom_bits are ignored) under settings varied one field at a
 * time, in the order partitioned, then (when the single-table path wins)
 * count_lanes, bloom_lanes, tiles_per_block, load_factor, bloom_bits,
 * aggregate, tails_overlap, keeping each change that makes the call at least
 * 1 % faster (best of `reps` runs per setting, reps >= 1).  The context keeps
 * the fastest setting, which is also written to *out; *report may be NULL.
 * A setting whose tables do not fit is skipped.  The reads are counted
 * several times: pass a representative read set of modest size. */
int kh_autotune(kh_ctx *ctx, const kh_reads *reads, const kh_params *params,
                const uint32_t *ks, int nk, void *hip_stream, int reps,
                kh_tuning *out, kh_tune_report *report);

/* kh_autotune with a persistent choice.  The text file cache_path holds one
 * line per tuned case, keyed by the device (architecture and compute-unit
 * count), the k set, the read and base counts, the Bloom setting and the
 * key-space part count.  If it holds the case, the context takes the stored
 * tuning without running any trial (*hit = 1, report zeroed); otherwise
 * kh_autotune runs and its choice is appended to the file (*hit = 0; a file
 * that cannot be written is not an error).  A later line for the same case
 * wins.  hit and report may be NULL. */
int kh_autotune_cached(kh_ctx *ctx, const kh_reads *reads, const kh_params *params,
                       const uint32_t *ks, int nk, void *hip_stream, int reps,
                       const char *cache_path, kh_tuning *out, kh_tune_report *report,
                       int *hit);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of read batches from many samples.
 *
 * A server owns its own context and a worker thread.  kh_server_submit
 * queues a batch of reads for a sample; the worker admits queued requests
 * (in arrival order) while fewer than max_active run and the device memory
 * in use plus the expected needs of running requests stays under 60 % of
 * the HBM budget (when nothing runs and no other sample is resident, the
 * oldest request runs regardless), and builds every launch from
 * chunks of several running requests,
 * so requests that arrive while others run share the next launches.  Each
 * sample keeps one table per k resident on the device (and its packed
 * reads, for the exact heavy-hitter recount) until kh_server_finalize turns
 * them into rows.  Counting is exact (no Bloom screen): the rows of a sample
 * are bit-identical to kh_count_multi_k on the union of its batches with
 * use_bloom = 0, whatever the arrival order and the mix (the table is a sum
 * of per-window updates; Section II-A, Use case 1).
 * ---------------------------------------------------------------------- */
typedef struct kh_server kh_server;

typedef struct {
  uint32_t max_active;  /* requests counted concurrently, default 16 */
  uint32_t queue_cap;   /* waiting requests before submit returns KH_EAGAIN,
                           default 1024 */
  int64_t chunk_reads;  /* reads of one request taken per round of a launch,
                           default 16384 */
  int64_t batch_bases;  /* bases per launch, default 32 Mi */
  uint32_t plain;       /* 1: first-in first-out, one request at a time, one
                           chunk per launch (the comparison mode) */
} kh_server_config;

void kh_server_default_config(kh_server_config *cfg);

/* Create a server on `device` counting at ks[0..nk) (nk <= 8) with the other
 * fields of params (use_bloom must be 0).  cfg may be NULL (defaults).
 * hbm_budget_bytes caps the device memory the server holds (0 = 85 % of the
 * device); a batch whose tables cannot grow within it fails with
 * KH_ENOMEM (its sample's finalize then reports the error). */
int kh_server_create(kh_server **out, int device, uint64_t hbm_budget_bytes,
                     const kh_params *params, const uint32_t *ks, int nk,
                     const kh_server_config *cfg);

/* Queue a batch of host reads for `sample`.  The caller keeps the three
 * arrays valid until the ticket completes.  KH_EAGAIN if the queue is full;
 * KH_EINVAL for device reads or bad offsets.  A sample's tables stay on the
 * device until it is finalized: when they fill the budget, queued batches
 * of other samples wait until the client finalizes samples. */
int kh_server_submit(kh_server *srv, uint64_t sample, const kh_reads *reads,
                     uint64_t *ticket);

/* Ticket state: *done = 1 once the batch has been counted at every k;
 * *latency_ms = completion - submission (-1 while running).  Returns the
 * batch's error code once done, KH_ENOTFOUND for an unknown ticket. */
int kh_server_poll(kh_server *srv, uint64_t ticket, int *done,
                   double *latency_ms);
int kh_server_wait(kh_server *srv, uint64_t ticket, double *latency_ms);

/* Wait for the sample's outstanding batches, then write its tables (one per
 * k, in the order of ks) to outs and release the sample.  KH_ENOTFOUND for an
 * unknown sample.  KH_ENOMEM if its rows may not fit the HBM budget while
 * other samples are resident: the sample stays and finalize can be called
 * again once other samples are finalized or tables freed.  The tables are
 * freed with kh_table_free. */
int kh_server_finalize(kh_server *srv, uint64_t sample, kh_table **outs);

/* [0] batches completed, [1] launches, [2] windows counted (all k),
 * [3] seconds the worker spent on launches, [4] most requests running at
 * once, [5] samples resident, [6] device bytes held, [7] table rehashes,
 * [8] windows replayed after their table filled up, [9] seconds of [3] in
 * upload and packing, [10] seconds of [3] growing tables, [11] most device
 * bytes held at once, [12] device allocations made, [13] seconds spent in
 * them, [14] launches that did not fit the budget and were retried with the
 * oldest request alone, [15] device bytes in use (held minus blocks free for
 * reuse), [16] device bytes reserved for admitted requests. */
int kh_server_stats(kh_server *srv, double out[17]);

/* Stop the worker (running batches finish; queued ones fail with
 * KH_EAGAIN) and release everything the server holds. */
int kh_server_destroy(kh_server *srv);

/* ------------------------------------------------------------------------
 * Counting without device allocation.
 *
 * For callers that cannot allocate device memory -- code around HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc -- this is
 * kh_count with every device buffer taken from a fixed scratch array of
 * KH_NOALLOC_SCRATCH_BYTES that the library's code object holds on each
 * device it runs on, until the process ends.  It needs no context, calls no
 * device allocator (neither HIP's nor any other library's) and frees
 * nothing; it runs on the calling thread's current device.
 * ---------------------------------------------------------------------- */
#define KH_NOALLOC_SCRATCH_BYTES (64ull << 20)
#define KH_NOALLOC_MAX_BASES (16ull << 20)

/* Count one read set at one k (params as for kh_count, with the library's
 * default tuning) and write the rows to the caller's device buffers: keys
 * max_rows*W uint64, counts max_rows uint32, ext max_rows*8 uint32, codes
 * max_rows*2 bytes, laid out as kh_table_export writes them.  The rows are
 * bit-identical to kh_count followed by kh_table_export.  *n_rows receives
 * the number of rows and *n_windows (may be NULL) the valid windows.
 *
 * The reads must be in device memory (on_device = 1) and hold at most
 * KH_NOALLOC_MAX_BASES bases (KH_EINVAL beyond).  KH_ENOMEM when the
 * k-mers (or, rarely, the sort of rows sharing their top 20 bases) need
 * more room than the scratch array holds -- roughly 1e6 distinct k-mers for
 * k <= 31, half that beyond.  KH_EOVERFLOW when the rows exceed max_rows:
 * *n_rows then holds the number needed and the call can be repeated with
 * larger buffers.  Other errors as for kh_count.
 *
 * Stream-ordered on `stream` and synchronous: it returns once its device
 * work has finished.  Calls on one device share that device's scratch
 * array; the library serialises them with a lock, so calls from several
 * threads wait for one another rather than overlap (work a caller enqueues
 * on other streams itself never touches the array).  Every buffer that must
 * start at zero is cleared by each call. */
int kh_count_noalloc(const kh_reads *reads, const kh_params *params, void *stream,
                     uint64_t *keys, uint32_t *counts, uint32_t *ext, uint8_t *codes,
                     int64_t max_rows, int64_t *n_rows, uint64_t *n_windows);

#ifdef __cplusplus
}
#endif
#endif /* KMERHIP_H */
