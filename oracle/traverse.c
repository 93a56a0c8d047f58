/*
 * CPU oracle for de Bruijn graph traversal -- TEST INFRASTRUCTURE ONLY.
 *
 * What it computes (paper Section II-C, de Bruijn graph traversal): the
 * vertices are the kept k-mers, each with its two-letter extension code; a
 * contig is a path of k-mers joined by unique high-quality extensions, and
 * fork / dead-end vertices end contigs.  The paper gives no algorithm for
 * this step beyond "traverse the graph", so the oracle states the result as
 * a definition and computes it with a plain sequential walk.
 *
 * Readings (the paper is silent on these):
 *  T1 An edge joins k-mer S to S' = S[1..k) + b when S's right code is the
 *     base b, S' (in canonical form) is a kept k-mer, and S''s left code is
 *     S[0] -- both ends must name each other (an edge is "mutual").  Codes of
 *     a k-mer read on its reverse strand swap sides and complement (F and X
 *     stay).  Left edges are the mirror image.
 *  T2 An edge from a k-mer to itself or to its own reverse complement is
 *     dropped (it cannot be walked as a simple path).
 *  T3 Every kept k-mer belongs to exactly one contig: a maximal path (a
 *     single k-mer with no edge is a contig of length k) or a cycle.
 *  T4 A path contig is written in the orientation whose sequence is
 *     lexicographically smaller (A<C<G<T) than its reverse complement.  A
 *     cycle is opened at its smallest k-mer (canonical key order) in its
 *     canonical orientation and written walking right, n k-mers giving
 *     k + n - 1 bases.
 *  T5 Contigs are listed by their smallest k-mer (ascending canonical key);
 *     each carries its number of k-mers and the sum of their counts (depth).
 *
 * Rows are taken in the library's export format (keys as W words, most
 * significant first, ascending; codes as two letters).  Lookups are binary
 * searches over the rows; nothing is hashed.
 *
 * Pins: the Python tests check this oracle against an independent brute
 * force (union of mutual edges over a Python dict) on random tiny tables,
 * against a circular genome (one cycle of known sequence), an error-free
 * linear genome (one contig equal to the genome) and a genome with a
 * planted repeat (four contigs worked out by hand).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static const char kLetters[4] = {'A', 'C', 'G', 'T'};

static char comp_letter(char c) {
  switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    default: return c; /* F and X stay */
  }
}

static int is_base(char c) { return c == 'A' || c == 'C' || c == 'G' || c == 'T'; }

static void revcomp_text(const char *s, uint32_t k, char *out) {
  for (uint32_t j = 0; j < k; j++) out[j] = comp_letter(s[k - 1 - j]);
}

typedef struct {
  uint32_t k;
  int64_t n;
  const char *text;      /* n rows of k letters (canonical keys, ascending) */
  const uint8_t *codes;  /* n * 2 */
} graph;

/* Row of a k-mer given in any orientation, or -1; *fwd = 1 if the text is
 * the row's canonical orientation. */
static int64_t find_row(const graph *g, const char *s, int *fwd) {
  char rc[128];
  revcomp_text(s, g->k, rc);
  const char *canon = s;
  *fwd = 1;
  if (memcmp(rc, s, g->k) < 0) {
    canon = rc;
    *fwd = 0;
  }
  int64_t lo = 0, hi = g->n;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    const int c = memcmp(g->text + (size_t)mid * g->k, canon, g->k);
    if (c < 0)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < g->n && memcmp(g->text + (size_t)lo * g->k, canon, g->k) == 0) return lo;
  return -1;
}

/* Left and right codes of a k-mer read in the given orientation (T1). */
static void oriented_codes(const graph *g, int64_t row, int fwd, char *left,
                           char *right) {
  const char l = (char)g->codes[2 * row], r = (char)g->codes[2 * row + 1];
  if (fwd) {
    *left = l;
    *right = r;
  } else {
    *left = comp_letter(r);
    *right = comp_letter(l);
  }
}

/* The k-mer after s (walking right), written into next; returns its row or
 * -1 if s has no mutual right edge (T1, T2).  `row` is s's own row. */
static int64_t step_right(const graph *g, const char *s, int64_t row, int fwd,
                          char *next) {
  char l, r;
  oriented_codes(g, row, fwd, &l, &r);
  if (!is_base(r)) return -1;
  memcpy(next, s + 1, g->k - 1);
  next[g->k - 1] = r;
  int nfwd;
  const int64_t nrow = find_row(g, next, &nfwd);
  if (nrow < 0 || nrow == row) return -1;
  char nl, nr;
  oriented_codes(g, nrow, nfwd, &nl, &nr);
  if (nl != s[0]) return -1;
  return nrow;
}

/* Mirror image: the k-mer before s. */
static int64_t step_left(const graph *g, const char *s, int64_t row, int fwd,
                         char *prev) {
  char l, r;
  oriented_codes(g, row, fwd, &l, &r);
  if (!is_base(l)) return -1;
  prev[0] = l;
  memcpy(prev + 1, s, g->k - 1);
  int pfwd;
  const int64_t prow = find_row(g, prev, &pfwd);
  if (prow < 0 || prow == row) return -1;
  char pl, pr;
  oriented_codes(g, prow, pfwd, &pl, &pr);
  if (pr != s[g->k - 1]) return -1;
  return prow;
}

typedef struct {
  char *seq;
  size_t len, cap;
} strbuf;

static int sb_push(strbuf *b, const char *s, size_t n) {
  if (b->len + n > b->cap) {
    size_t c = b->cap ? 2 * b->cap : 1024;
    while (c < b->len + n) c *= 2;
    char *p = (char *)realloc(b->seq, c);
    if (!p) return -1;
    b->seq = p;
    b->cap = c;
  }
  memcpy(b->seq + b->len, s, n);
  b->len += n;
  return 0;
}

int oracle_traverse(const uint64_t *keys, const uint32_t *counts,
                    const uint8_t *codes, int64_t n, uint32_t k,
                    oracle_contigs **out) {
  if (!out || k < 1 || k > 127 || n < 0 || (n > 0 && (!keys || !counts || !codes)))
    return -1;
  *out = NULL;
  const uint32_t W = (k + 31) / 32;
  char *text = (char *)malloc((size_t)(n > 0 ? n : 1) * k);
  uint8_t *visited = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
  oracle_contigs *c = (oracle_contigs *)calloc(1, sizeof *c);
  int64_t cap = 1024;
  if (c) {
    c->offsets = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap + 1));
    c->n_kmers = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    c->depth = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)cap);
    c->cycle = (uint8_t *)malloc((size_t)cap);
  }
  strbuf all = {0}, one = {0};
  char *cur = (char *)malloc(k), *nxt = (char *)malloc(k), *rc = NULL;
  int rcode = -1;
  if (!text || !visited || !c || !c->offsets || !c->n_kmers || !c->depth ||
      !c->cycle || !cur || !nxt)
    goto done;
  for (int64_t i = 0; i < n; i++)
    for (uint32_t j = 0; j < k; j++) {
      const uint32_t bit = 2 * (k - 1 - j);
      text[(size_t)i * k + j] = kLetters[(keys[(size_t)i * W + W - 1 - bit / 64] >> (bit % 64)) & 3];
    }
  graph g = {k, n, text, codes};
  c->offsets[0] = 0;
  for (int64_t i = 0; i < n; i++) {
    if (visited[i]) continue;
    /* walk left from row i (canonical orientation) to the start of its path,
       or around to i itself if it lies on a cycle */
    memcpy(cur, text + (size_t)i * k, k);
    int64_t row = i;
    int fwd = 1, cyc = 0;
    for (int64_t steps = 0;; steps++) {
      if (steps > n) goto done; /* cannot happen: components are paths or cycles */
      const int64_t prow = step_left(&g, cur, row, fwd, nxt);
      if (prow < 0) break;
      if (prow == i) {
        cyc = 1;
        break;
      }
      int f;
      find_row(&g, nxt, &f);
      memcpy(cur, nxt, k);
      row = prow;
      fwd = f;
    }
    if (cyc) { /* T4: open the cycle at row i, canonical orientation */
      memcpy(cur, text + (size_t)i * k, k);
      row = i;
      fwd = 1;
    }
    /* walk right, writing the contig */
    one.len = 0;
    if (sb_push(&one, cur, k)) goto done;
    int64_t nk = 0;
    uint64_t depth = 0;
    for (;;) {
      visited[row] = 1;
      nk++;
      depth += counts[row];
      const int64_t nrow = step_right(&g, cur, row, fwd, nxt);
      if (nrow < 0 || (cyc && nrow == i)) break; /* path end, or the cycle closed */
      if (nk > n) goto done; /* cannot happen for a simple path: refuse to loop */
      int f;
      find_row(&g, nxt, &f);
      if (sb_push(&one, nxt + k - 1, 1)) goto done;
      memcpy(cur, nxt, k);
      row = nrow;
      fwd = f;
    }
    if (!cyc) { /* T4: the smaller of the path and its reverse complement */
      free(rc);
      rc = (char *)malloc(one.len);
      if (!rc) goto done;
      revcomp_text(one.seq, (uint32_t)one.len, rc);
      if (memcmp(rc, one.seq, one.len) < 0) memcpy(one.seq, rc, one.len);
    }
    if (c->n_contigs == cap) {
      cap *= 2;
      int64_t *o = (int64_t *)realloc(c->offsets, sizeof(int64_t) * (size_t)(cap + 1));
      if (o) c->offsets = o;
      int64_t *m = (int64_t *)realloc(c->n_kmers, sizeof(int64_t) * (size_t)cap);
      if (m) c->n_kmers = m;
      uint64_t *d = (uint64_t *)realloc(c->depth, sizeof(uint64_t) * (size_t)cap);
      if (d) c->depth = d;
      uint8_t *y = (uint8_t *)realloc(c->cycle, (size_t)cap);
      if (y) c->cycle = y;
      if (!o || !m || !d || !y) goto done;
    }
    if (sb_push(&all, one.seq, one.len)) goto done;
    c->n_kmers[c->n_contigs] = nk;
    c->depth[c->n_contigs] = depth;
    c->cycle[c->n_contigs] = (uint8_t)cyc;
    c->n_contigs++;
    c->offsets[c->n_contigs] = (int64_t)all.len;
  }
  c->total_len = (int64_t)all.len;
  c->seq = all.seq;
  all.seq = NULL;
  rcode = 0;
done:
  free(text);
  free(visited);
  free(cur);
  free(nxt);
  free(rc);
  free(all.seq);
  free(one.seq);
  if (rcode == 0) {
    *out = c;
  } else if (c) {
    oracle_contigs_free(c);
  }
  return rcode;
}

void oracle_contigs_free(oracle_contigs *c) {
  if (!c) return;
  free(c->seq);
  free(c->offsets);
  free(c->n_kmers);
  free(c->depth);
  free(c->cycle);
  free(c);
}
