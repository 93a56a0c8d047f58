/*
 * CPU oracle for read localisation -- TEST INFRASTRUCTURE ONLY.
 *
 * What it computes (paper Section II, the read localisation subsection):
 * after the first iteration, reads that come from the same contig region are
 * brought together, so that in later iterations the occurrences of a k-mer
 * arrive close together and the counting table's updates hit in cache.  The
 * paper assigns each read to the contig it aligns to; alignment is not part
 * of this library, so the contig is found through the read's k-mers.
 *
 * Readings (the paper leaves these open):
 *  L1 A read's anchor is the first of its windows, in read order, that holds
 *     k bases of A/C/G/T (lowercase counts as the base) and whose canonical
 *     k-mer lies in a contig; the read's contig is that contig's index.
 *  L2 Reads are ordered by contig index, stably (reads of one contig keep
 *     their input order); reads without an anchor follow all others, in
 *     input order.
 *  L3 Localisation permutes reads only: every table counted from the
 *     permuted reads equals the table of the input (Section II-A, Use
 *     case 1: the result does not depend on the order of insertions).
 *
 * Pins: the Python tests check this oracle against an independent brute
 * force (Python dicts) on random reads and contigs, and against a closed
 * form: reads tiled error-free from several genomes, shuffled together,
 * come back grouped genome by genome in their shuffled order, with reads of
 * foreign sequence last.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static char lz_up(char c) { return (c >= 'a' && c <= 'z') ? (char)(c - 32) : c; }
static int lz_acgt(char c) { return c == 'A' || c == 'C' || c == 'G' || c == 'T'; }
static char lz_comp(char c) {
  switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    default: return 'A';
  }
}

typedef struct {
  const char *key; /* k letters, canonical */
  int64_t contig;
} lref;

static uint32_t lz_k;
static int cmp_lref(const void *a, const void *b) {
  const lref *x = (const lref *)a, *y = (const lref *)b;
  const int c = memcmp(x->key, y->key, lz_k);
  if (c) return c;
  return x->contig < y->contig ? -1 : x->contig > y->contig; /* a shared k-mer: first contig */
}

static void lz_canonical(const char *w, uint32_t k, char *rc, char *out) {
  for (uint32_t j = 0; j < k; j++) rc[j] = lz_comp(w[k - 1 - j]);
  memcpy(out, memcmp(rc, w, k) < 0 ? rc : w, k);
}

int oracle_localize(const uint8_t *seq, const int64_t *offsets, int64_t n_reads, uint32_t k,
                    const char *cseq, const int64_t *coff, int64_t n_contigs,
                    int64_t *order) {
  if (k < 1 || k > 127 || n_reads < 0 || n_contigs < 0 || !order ||
      (n_reads > 0 && (!seq || !offsets)) || (n_contigs > 0 && (!cseq || !coff)))
    return -1;
  int64_t nref = 0;
  for (int64_t c = 0; c < n_contigs; c++) {
    const int64_t len = coff[c + 1] - coff[c];
    if (len >= (int64_t)k) nref += len - k + 1;
  }
  int rcode = -1;
  lref *refs = (lref *)malloc(sizeof(lref) * (size_t)(nref > 0 ? nref : 1));
  char *store = (char *)malloc((size_t)(nref > 0 ? nref : 1) * k);
  int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_reads > 0 ? n_reads : 1));
  int64_t *start = (int64_t *)calloc((size_t)n_contigs + 2, sizeof(int64_t));
  char *w = (char *)malloc(k), *rc = (char *)malloc(k), *canon = (char *)malloc(k);
  if (!refs || !store || !key || !start || !w || !rc || !canon) goto done;
  /* ---- contig k-mers (canonical) with their contig */
  {
    int64_t m = 0;
    for (int64_t c = 0; c < n_contigs; c++)
      for (int64_t p = coff[c]; p + (int64_t)k <= coff[c + 1]; p++) {
        int ok = 1;
        for (uint32_t j = 0; j < k; j++) {
          w[j] = lz_up(cseq[p + j]);
          ok = ok && lz_acgt(w[j]);
        }
        if (!ok) continue;
        char *dst = store + (size_t)m * k;
        lz_canonical(w, k, rc, dst);
        refs[m].key = dst;
        refs[m].contig = c;
        m++;
      }
    nref = m;
    lz_k = k;
    qsort(refs, (size_t)nref, sizeof(lref), cmp_lref);
  }
  /* ---- anchor of every read (L1) */
  for (int64_t r = 0; r < n_reads; r++) {
    key[r] = n_contigs; /* no anchor: after every contig */
    const int64_t o = offsets[r], len = offsets[r + 1] - o;
    for (int64_t p = 0; p + (int64_t)k <= len; p++) {
      int ok = 1;
      for (uint32_t j = 0; j < k && ok; j++) {
        w[j] = lz_up((char)seq[o + p + j]);
        ok = lz_acgt(w[j]);
      }
      if (!ok) continue;
      lz_canonical(w, k, rc, canon);
      int64_t lo = 0, hi = nref;
      while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (memcmp(refs[mid].key, canon, k) < 0) lo = mid + 1; else hi = mid;
      }
      if (lo < nref && memcmp(refs[lo].key, canon, k) == 0) {
        key[r] = refs[lo].contig;
        break;
      }
    }
  }
  /* ---- stable counting sort by contig (L2) */
  for (int64_t r = 0; r < n_reads; r++) start[key[r] + 1]++;
  for (int64_t c = 0; c <= n_contigs; c++) start[c + 1] += start[c];
  for (int64_t r = 0; r < n_reads; r++) order[start[key[r]]++] = r;
  rcode = 0;
done:
  free(refs);
  free(store);
  free(key);
  free(start);
  free(w);
  free(rc);
  free(canon);
  return rcode;
}
