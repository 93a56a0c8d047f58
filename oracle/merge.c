/*
 * CPU oracle for merging a k-mer table with the k-mers of earlier contigs
 * -- TEST INFRASTRUCTURE ONLY.
 *
 * What it computes (paper Section II, Algorithm 1's Merge step, and the
 * subsection on merging k-mer sets): the k-mers of the contigs assembled
 * with a smaller k are taken as error-free (k+s)-mers with unique
 * high-quality extensions and merged into the (k+s)-mer table of the
 * reads, a k-mer present in both kept once.
 *
 * Readings (the paper leaves these open):
 *  M1 The contig k-mers are every window of every contig that holds only
 *     A/C/G/T, in canonical form (the same canonical rule as the table);
 *     the neighbouring contig bases are its extensions, swapped and
 *     complemented when the reverse complement is the key.
 *  M2 A k-mer that is already a row keeps that row unchanged (the reads'
 *     k-mers are stored first; storing the same key again finds it).
 *  M3 A k-mer found only in the contigs becomes a row with count 0, no
 *     tallies, and per side the code: the neighbouring base when every
 *     occurrence has one and they all agree; 'X' when no occurrence has
 *     one; 'F' otherwise.
 *  M4 Rows stay in ascending key order.
 *
 * Pins: the Python tests check this oracle against an independent brute
 * force (Python dicts and sets) on random tables and contigs, and against
 * closed forms: merging a contig into an empty table and walking the result
 * gives the contig back; merging contigs whose k-mers are all rows changes
 * nothing.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static char up(char c) { return (c >= 'a' && c <= 'z') ? (char)(c - 32) : c; }
static int is_acgt(char c) { return c == 'A' || c == 'C' || c == 'G' || c == 'T'; }
static char comp_base(char c) {
  switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    default: return c;
  }
}
static int letter_value(char c) { return c == 'A' ? 0 : c == 'C' ? 1 : c == 'G' ? 2 : 3; }

typedef struct {
  char *key; /* k letters, canonical */
  char left, right; /* neighbouring base or 0 */
} crec;

static uint32_t g_k;
static int cmp_crec(const void *a, const void *b) {
  return memcmp(((const crec *)a)->key, ((const crec *)b)->key, g_k);
}

static void to_text(const uint64_t *w, uint32_t k, uint32_t W, char *out) {
  static const char L[4] = {'A', 'C', 'G', 'T'};
  for (uint32_t j = 0; j < k; j++) {
    const uint32_t bit = 2 * (k - 1 - j);
    out[j] = L[(w[W - 1 - bit / 64] >> (bit % 64)) & 3];
  }
}

static void to_words(const char *s, uint32_t k, uint32_t W, uint64_t *w) {
  memset(w, 0, sizeof(uint64_t) * W);
  for (uint32_t j = 0; j < k; j++) {
    const uint32_t bit = 2 * (k - 1 - j);
    w[W - 1 - bit / 64] |= (uint64_t)letter_value(s[j]) << (bit % 64);
  }
}

/* side code by M3 from: any occurrence lacking a neighbour, the set of
 * neighbouring bases seen */
static uint8_t side_code(int none, int seen_mask) {
  int nb = 0, which = 0;
  for (int b = 0; b < 4; b++)
    if (seen_mask & (1 << b)) {
      nb++;
      which = b;
    }
  if (nb == 0) return 'X';
  if (nb == 1 && !none) return (uint8_t)"ACGT"[which];
  return 'F';
}

int oracle_merge(const uint64_t *keys, const uint32_t *counts, const uint32_t *ext,
                 const uint8_t *codes, int64_t n, uint32_t k, const char *cseq,
                 const int64_t *coff, int64_t n_contigs, oracle_table **out) {
  if (!out || k < 1 || k > 127 || n < 0 || n_contigs < 0 ||
      (n > 0 && (!keys || !counts || !ext || !codes)) || (n_contigs > 0 && (!cseq || !coff)))
    return -1;
  *out = NULL;
  const uint32_t W = (k + 31) / 32;
  g_k = k;
  /* ---- records of every contig window (M1) */
  int64_t nrec = 0;
  for (int64_t c = 0; c < n_contigs; c++) {
    const int64_t len = coff[c + 1] - coff[c];
    if (len >= (int64_t)k) nrec += len - k + 1;
  }
  crec *rec = (crec *)malloc(sizeof(crec) * (size_t)(nrec > 0 ? nrec : 1));
  char *store = (char *)malloc((size_t)(nrec > 0 ? nrec : 1) * k);
  char *text = (char *)malloc((size_t)(n > 0 ? n : 1) * k);
  char *w = (char *)malloc(k), *rc = (char *)malloc(k);
  oracle_table *t = (oracle_table *)calloc(1, sizeof *t);
  int rcode = -1;
  if (!rec || !store || !text || !w || !rc || !t) goto done;
  int64_t m = 0;
  for (int64_t c = 0; c < n_contigs; c++) {
    const char *s = cseq + coff[c];
    const int64_t len = coff[c + 1] - coff[c];
    for (int64_t p = 0; p + (int64_t)k <= len; p++) {
      int ok = 1;
      for (uint32_t j = 0; j < k; j++) {
        w[j] = up(s[p + j]);
        ok = ok && is_acgt(w[j]);
      }
      if (!ok) continue;
      const char l = (p > 0 && is_acgt(up(s[p - 1]))) ? up(s[p - 1]) : 0;
      const char r = (p + (int64_t)k < len && is_acgt(up(s[p + k]))) ? up(s[p + k]) : 0;
      for (uint32_t j = 0; j < k; j++) rc[j] = comp_base(w[k - 1 - j]);
      crec *x = &rec[m];
      x->key = store + (size_t)m * k;
      if (memcmp(rc, w, k) < 0) {
        memcpy(x->key, rc, k);
        x->left = r ? comp_base(r) : 0;
        x->right = l ? comp_base(l) : 0;
      } else {
        memcpy(x->key, w, k);
        x->left = l;
        x->right = r;
      }
      m++;
    }
  }
  qsort(rec, (size_t)m, sizeof(crec), cmp_crec);
  /* ---- table keys as text for lookups */
  for (int64_t i = 0; i < n; i++) to_text(keys + (size_t)i * W, k, W, text + (size_t)i * k);
  /* ---- new rows: contig k-mers that are not rows (M2, M3) */
  int64_t n_new = 0;
  char *new_keys = (char *)malloc((size_t)(m > 0 ? m : 1) * k);
  uint8_t *new_codes = (uint8_t *)malloc((size_t)(m > 0 ? m : 1) * 2);
  if (!new_keys || !new_codes) {
    free(new_keys);
    free(new_codes);
    goto done;
  }
  for (int64_t a = 0; a < m;) {
    int64_t b = a;
    int lnone = 0, rnone = 0, lmask = 0, rmask = 0;
    while (b < m && memcmp(rec[b].key, rec[a].key, k) == 0) {
      if (rec[b].left) lmask |= 1 << letter_value(rec[b].left); else lnone = 1;
      if (rec[b].right) rmask |= 1 << letter_value(rec[b].right); else rnone = 1;
      b++;
    }
    /* present in the table? binary search over the sorted row keys */
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (memcmp(text + (size_t)mid * k, rec[a].key, k) < 0) lo = mid + 1; else hi = mid;
    }
    const int present = lo < n && memcmp(text + (size_t)lo * k, rec[a].key, k) == 0;
    if (!present) {
      memcpy(new_keys + (size_t)n_new * k, rec[a].key, k);
      new_codes[2 * n_new] = side_code(lnone, lmask);
      new_codes[2 * n_new + 1] = side_code(rnone, rmask);
      n_new++;
    }
    a = b;
  }
  /* ---- merge the two sorted lists (M4) */
  const int64_t total = n + n_new;
  t->k = k;
  t->W = W;
  t->n_rows = total;
  t->keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(total > 0 ? total : 1) * W);
  t->counts = (uint32_t *)calloc((size_t)(total > 0 ? total : 1), sizeof(uint32_t));
  t->ext = (uint32_t *)calloc((size_t)(total > 0 ? total : 1) * 8, sizeof(uint32_t));
  t->codes = (uint8_t *)malloc((size_t)(total > 0 ? total : 1) * 2);
  if (!t->keys || !t->counts || !t->ext || !t->codes) {
    free(new_keys);
    free(new_codes);
    goto done;
  }
  int64_t i = 0, j = 0, o = 0;
  while (i < n || j < n_new) {
    const int take_old =
        j >= n_new || (i < n && memcmp(text + (size_t)i * k, new_keys + (size_t)j * k, k) < 0);
    if (take_old) {
      memcpy(t->keys + (size_t)o * W, keys + (size_t)i * W, sizeof(uint64_t) * W);
      t->counts[o] = counts[i];
      memcpy(t->ext + (size_t)o * 8, ext + (size_t)i * 8, sizeof(uint32_t) * 8);
      t->codes[2 * o] = codes[2 * i];
      t->codes[2 * o + 1] = codes[2 * i + 1];
      i++;
    } else {
      to_words(new_keys + (size_t)j * k, k, W, t->keys + (size_t)o * W);
      t->codes[2 * o] = new_codes[2 * j];
      t->codes[2 * o + 1] = new_codes[2 * j + 1];
      j++;
    }
    o++;
  }
  free(new_keys);
  free(new_codes);
  rcode = 0;
done:
  free(rec);
  free(store);
  free(text);
  free(w);
  free(rc);
  if (rcode == 0) {
    *out = t;
  } else if (t) {
    oracle_free(t);
  }
  return rcode;
}
