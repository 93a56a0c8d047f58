/*
 * CPU oracle for k-mer analysis -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code.  The GPU library never links, loads or calls it, and the
 * two share no source, header, table or helper.
 *
 * What it computes (paper Section II-B, "K-mer Analysis using Distributed
 * Histograms"): every read is split into k-mers overlapping by k-1 bases; each
 * k-mer is counted, the bases immediately before and after it in the read are
 * tallied as its left/right extensions, and k-mers whose count reaches the
 * threshold are kept.  Section II-C gives the output form (the k-mer as key
 * plus a two-letter extension code) and the depth-adaptive rule that decides
 * whether an extension is unique.  Section II-A (Use case 1) states that the
 * final table does not depend on insertion order, so the oracle emits its
 * rows in ascending key order.
 *
 * Readings where the paper is silent (canonical form, 2-bit order, quality
 * cutoff, non-ACGT bases, tie and dead-end letters) are listed in the
 * comments of oracle.c next to the code that applies them.
 *
 * Pins: the Python test suite checks this oracle against an independent brute
 * force (tiny inputs, exhaustive short reads), closed-form window totals,
 * reverse-complement and order invariance, hand-built special cases and
 * hand-built classifier vectors.  No function here is "parity unpinned".
 */
#ifndef KMER_ORACLE_H
#define KMER_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  uint32_t k;           /* k-mer length, 1..127 */
  uint32_t min_count;   /* keep k-mers with count >= min_count */
  int32_t qual_offset;  /* Phred encoding offset, 33 */
  int32_t qual_cutoff;  /* an extension base counts iff Phred >= cutoff */
  uint32_t t_min_ext;   /* fewer observations than this: dead end 'X' */
  uint32_t t_base;      /* floor of the contradiction threshold */
  uint32_t err_ppm;     /* error-model slope e, parts per million */
} oracle_params;

typedef struct {
  uint32_t k, W;            /* W = ceil(k / 32) key words per row */
  int64_t n_rows;           /* rows kept (count >= min_count) */
  uint64_t *keys;           /* n_rows * W, most significant word first */
  uint32_t *counts;         /* n_rows */
  uint32_t *ext;            /* n_rows * 8: left A,C,G,T then right A,C,G,T */
  uint8_t *codes;           /* n_rows * 2: left, right in {A,C,G,T,F,X} */
  /* totals before the count threshold */
  uint64_t n_windows;       /* valid windows = sum of all counts */
  uint64_t n_distinct;      /* distinct canonical k-mers */
  uint64_t sum_left;        /* sum of all left extension tallies */
  uint64_t sum_right;       /* sum of all right extension tallies */
} oracle_table;

/* Full table of one read set.  Returns 0, or -1 on bad arguments / memory. */
int oracle_count(const uint8_t *seq, const uint8_t *qual,
                 const int64_t *offsets, int64_t n_reads,
                 const oracle_params *p, oracle_table **out);

/* Same, restricted to the k-mers whose shard hash is s (mod S); see
 * oracle_shard_of.  Uses OpenMP over reads for large inputs. */
int oracle_count_shard(const uint8_t *seq, const uint8_t *qual,
                       const int64_t *offsets, int64_t n_reads,
                       const oracle_params *p, uint64_t S, uint64_t s,
                       oracle_table **out);

/* Records of the given query keys (nq keys of W words each), before the
 * threshold: counts[q] and ext[q*8 .. q*8+8).  Unseen keys get zeros. */
int oracle_count_keys(const uint8_t *seq, const uint8_t *qual,
                      const int64_t *offsets, int64_t n_reads,
                      const oracle_params *p, const uint64_t *qkeys,
                      int64_t nq, uint64_t *counts, uint64_t *ext);

/* Shard hash of a W-word key: h = 0; h = mix64(h ^ word) for each word from
 * the most significant; shard = h mod S (mix64 = SplitMix64 output step). */
uint64_t oracle_shard_of(const uint64_t *key, uint32_t W, uint64_t S);

/* Extension letter for one side: c = tallies of A,C,G,T, depth = k-mer count. */
uint8_t oracle_classify_side(const uint64_t c[4], uint64_t depth,
                             const oracle_params *p);

void oracle_free(oracle_table *t);

/* OpenMP threads of the calling thread's later parallel regions. */
void oracle_set_threads(int n);

/* ---- de Bruijn graph traversal (traverse.c) ------------------------------
 * Contigs of a k-mer table (paper Section II-C): maximal paths of k-mers
 * joined by mutual unique extensions; readings T1-T5 in traverse.c. */
typedef struct {
  int64_t n_contigs;
  int64_t total_len;   /* bases over all contigs */
  char *seq;           /* concatenated contig sequences, ASCII */
  int64_t *offsets;    /* n_contigs + 1 */
  int64_t *n_kmers;    /* k-mers per contig */
  uint64_t *depth;     /* sum of the k-mers' counts */
  uint8_t *cycle;      /* 1 for a cycle */
} oracle_contigs;

/* Rows as exported (keys n * W ascending, counts n, codes n * 2).  Returns 0,
 * or -1 on bad arguments / memory. */
int oracle_traverse(const uint64_t *keys, const uint32_t *counts,
                    const uint8_t *codes, int64_t n, uint32_t k,
                    oracle_contigs **out);
void oracle_contigs_free(oracle_contigs *c);

/* ---- merging earlier contigs' k-mers (merge.c) ------------------------------
 * Rows of a table (as exported) merged with every k-mer of the given contigs
 * (ASCII, back to back, offsets n_contigs + 1); readings M1-M4 in merge.c.
 * The result's totals (n_windows ...) are left 0.  Returns 0 or -1. */
int oracle_merge(const uint64_t *keys, const uint32_t *counts, const uint32_t *ext,
                 const uint8_t *codes, int64_t n, uint32_t k, const char *cseq,
                 const int64_t *coffsets, int64_t n_contigs, oracle_table **out);

/* ---- iterative graph pruning (prune.c) -------------------------------------
 * Algorithm 2 over a contig set (ASCII A/C/G/T, back to back, offsets
 * n_contigs + 1; depth = sum of each contig's k-mer counts) that shares no
 * k-mer between contigs; readings P1-P7 in prune.c.  removed_at[c] (caller
 * allocates n_contigs) = the sweep that removed contig c, or -1; *sweeps =
 * sweeps run.  alpha in [1e-3, 1e3], beta in [0, 1e6].  Returns 0 or -1. */
int oracle_prune(const char *cseq, const int64_t *coffsets, const uint64_t *depth,
                 int64_t n_contigs, uint32_t k, double alpha, double beta,
                 int32_t *removed_at, int64_t *sweeps);

/* ---- read localisation (localize.c) ----------------------------------------
 * Order of the reads (seq/offsets as for oracle_count) grouped by the contig
 * holding each read's first k-mer found in a contig (ASCII contigs back to
 * back, offsets n_contigs + 1); readings L1-L3 in localize.c.  order (caller
 * allocates n_reads) receives read indices.  Returns 0 or -1. */
int oracle_localize(const uint8_t *seq, const int64_t *offsets, int64_t n_reads, uint32_t k,
                    const char *cseq, const int64_t *coffsets, int64_t n_contigs,
                    int64_t *order);

#ifdef __cplusplus
}
#endif
#endif
