/*
 * Drives every entry point of the CPU oracle on small random inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitized.py compiles and runs it).  It checks no
 * result: the pin suites do that.  Its job is to make any out-of-bounds
 * access, leak or undefined operation in the oracle's C code abort the run.
 *
 * Inputs: a random genome; reads cut from it on both strands with
 * substitutions, N and lowercase bases, random qualities, some shorter than
 * k and some empty; k from 1 to 127.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

static uint64_t g_state = 0x1809070140ull;

static uint64_t next_u64(void) { /* SplitMix64 */
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

static uint32_t below(uint32_t n) { return (uint32_t)(next_u64() % n); }

typedef struct {
  uint8_t *seq, *qual;
  int64_t *off;
  int64_t n_reads;
} reads;

static reads make_reads(const char *genome, int64_t glen, int64_t n_reads) {
  reads r;
  r.n_reads = n_reads;
  r.off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_reads + 1));
  int64_t total = 0;
  int64_t *len = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_reads);
  for (int64_t i = 0; i < n_reads; i++) {
    len[i] = (i % 17 == 0) ? 0 : (int64_t)below(160);
    if (len[i] > glen) len[i] = glen;
    total += len[i];
  }
  r.seq = (uint8_t *)malloc((size_t)(total ? total : 1));
  r.qual = (uint8_t *)malloc((size_t)(total ? total : 1));
  static const char comp[256] = {['A'] = 'T', ['C'] = 'G', ['G'] = 'C', ['T'] = 'A'};
  int64_t p = 0;
  r.off[0] = 0;
  for (int64_t i = 0; i < n_reads; i++) {
    const int64_t start = len[i] ? (int64_t)below((uint32_t)(glen - len[i] + 1)) : 0;
    const int rev = (int)below(2);
    for (int64_t j = 0; j < len[i]; j++) {
      char b = rev ? comp[(unsigned char)genome[start + len[i] - 1 - j]] : genome[start + j];
      const uint32_t e = below(1000);
      if (e < 5) b = "ACGT"[below(4)];
      else if (e < 8) b = 'N';
      else if (e < 12) b = (char)(b | 0x20); /* lowercase */
      r.seq[p] = (uint8_t)b;
      r.qual[p] = (uint8_t)(33 + 2 + below(40));
      p++;
    }
    r.off[i + 1] = p;
  }
  free(len);
  return r;
}

static void free_reads(reads *r) {
  free(r->seq);
  free(r->qual);
  free(r->off);
}

static int run_k(const reads *r, uint32_t k) {
  oracle_params p = {k, 2, 33, 20, 2, 1, 5000};
  if (k < 9) p.min_count = 1;
  oracle_table *t = NULL;
  if (oracle_count(r->seq, r->qual, r->off, r->n_reads, &p, &t)) return 1;

  /* shards and query keys */
  for (uint64_t s = 0; s < 3; s++) {
    oracle_table *ts = NULL;
    if (oracle_count_shard(r->seq, r->qual, r->off, r->n_reads, &p, 3, s, &ts)) return 2;
    oracle_free(ts);
  }
  const int64_t nq = t->n_rows < 50 ? t->n_rows : 50;
  uint64_t *counts = (uint64_t *)calloc((size_t)(nq ? nq : 1), sizeof(uint64_t));
  uint64_t *ext = (uint64_t *)calloc((size_t)(nq ? nq : 1) * 8, sizeof(uint64_t));
  if (oracle_count_keys(r->seq, r->qual, r->off, r->n_reads, &p, t->keys, nq, counts, ext))
    return 3;
  free(counts);
  free(ext);

  /* contigs of the table, merged back, pruned, used to localise the reads */
  oracle_contigs *c = NULL;
  if (oracle_traverse(t->keys, t->counts, t->codes, t->n_rows, k, &c)) return 4;
  oracle_table *m = NULL;
  if (oracle_merge(t->keys, t->counts, t->ext, t->codes, t->n_rows, k, c->seq, c->offsets,
                   c->n_contigs, &m))
    return 5;
  oracle_free(m);
  int32_t *removed = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c->n_contigs + 1));
  int64_t sweeps = 0;
  if (oracle_prune(c->seq, c->offsets, c->depth, c->n_contigs, k, 0.1, 0.2, removed,
                   &sweeps))
    return 6;
  free(removed);
  int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(r->n_reads + 1));
  if (oracle_localize(r->seq, r->off, r->n_reads, k, c->seq, c->offsets, c->n_contigs,
                      order))
    return 7;
  free(order);
  printf("k=%u rows=%lld contigs=%lld sweeps=%lld\n", k, (long long)t->n_rows,
         (long long)c->n_contigs, (long long)sweeps);
  oracle_contigs_free(c);
  oracle_free(t);
  return 0;
}

int main(void) {
  const int64_t glen = 3000;
  char *genome = (char *)malloc((size_t)glen + 1);
  for (int64_t i = 0; i < glen; i++) genome[i] = "ACGT"[below(4)];
  genome[glen] = 0;
  reads r = make_reads(genome, glen, 600);
  static const uint32_t ks[] = {1, 3, 5, 21, 31, 33, 63, 65, 77, 99, 127};
  for (size_t i = 0; i < sizeof ks / sizeof ks[0]; i++) {
    const int rc = run_k(&r, ks[i]);
    if (rc) {
      printf("oracle call %d failed at k=%u\n", rc, ks[i]);
      return 1;
    }
  }
  /* no reads at all */
  oracle_params p = {21, 2, 33, 20, 2, 1, 5000};
  int64_t zero = 0;
  oracle_table *t = NULL;
  if (oracle_count(NULL, NULL, &zero, 0, &p, &t)) return 1;
  oracle_free(t);
  free_reads(&r);
  free(genome);
  printf("sanitized oracle run ok\n");
  return 0;
}
