/*
 * CPU oracle for k-mer analysis -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Deliberately plain: every valid window of every read becomes one record
 * (canonical k-mer as ASCII text, left letter, right letter); the records are
 * sorted with the C library's qsort and equal keys are summed.  A sorted array
 * grouped by key is the ordered map over canonical k-mers.  No bit packing,
 * hashing, rolling or blocking is used to find or count k-mers; 2-bit words
 * are produced only at the very end, to export rows in the library's format.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- letters ----------------------------------------------------------- */

/* Reading of the paper's alphabet (Section II: reads are strings over
 * A, C, G, T).  Lowercase a/c/g/t are the same bases.  Any other byte (N,
 * IUPAC codes, ...) is not a base: a window that contains one is not a
 * k-mer, and such a neighbour is not an extension.  Returns 0 for those. */
static uint8_t as_base(uint8_t c) {
  switch (c) {
    case 'A': case 'a': return 'A';
    case 'C': case 'c': return 'C';
    case 'G': case 'g': return 'G';
    case 'T': case 't': return 'T';
    default: return 0;
  }
}

/* Watson-Crick complement; 0 ("no extension") stays 0. */
static uint8_t complement(uint8_t b) {
  switch (b) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    default: return 0;
  }
}

/* Position of a base in A < C < G < T. */
static int letter_index(uint8_t b) {
  switch (b) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    default: return 3;
  }
}

/* ---- one window -------------------------------------------------------- */

/* Reading of "high quality extension" for a single observation: the
 * neighbour base counts toward the k-mer's extension tally only when its
 * Phred score (byte - qual_offset) is at least qual_cutoff. */
static int good_quality(uint8_t qbyte, const oracle_params *p) {
  return (int)qbyte - p->qual_offset >= p->qual_cutoff;
}

/* Window s[i .. i+k) of a read of length len (Section II-B: k-mers overlap
 * by k-1 bases, extensions are the bases just before and after).  Writes the
 * canonical k-mer to key (k letters) and the extension letters seen from
 * the canonical strand to *L and *R (0 = none).  Returns 0 if the window
 * holds a non-base.
 *
 * Canonical form (reading: a k-mer and its reverse complement are the same
 * vertex; the representative is the lexicographically smaller of the two,
 * with A < C < G < T).  When the reverse complement is chosen, reading the
 * read on the other strand swaps the sides and complements the letters:
 * the new left is the complement of the old right and vice versa. */
static int window_record(const uint8_t *s, const uint8_t *q, int64_t len,
                         int64_t i, const oracle_params *p, uint8_t *fwd,
                         uint8_t *rc, uint8_t *key, uint8_t *L, uint8_t *R) {
  const int64_t k = p->k;
  for (int64_t j = 0; j < k; j++) {
    fwd[j] = as_base(s[i + j]);
    if (!fwd[j]) return 0;
  }
  uint8_t fl = 0, fr = 0;
  if (i >= 1 && as_base(s[i - 1]) && good_quality(q[i - 1], p))
    fl = as_base(s[i - 1]);
  if (i + k < len && as_base(s[i + k]) && good_quality(q[i + k], p))
    fr = as_base(s[i + k]);
  for (int64_t j = 0; j < k; j++) rc[j] = complement(fwd[k - 1 - j]);
  if (memcmp(fwd, rc, (size_t)k) <= 0) {
    memcpy(key, fwd, (size_t)k);
    *L = fl;
    *R = fr;
  } else {
    memcpy(key, rc, (size_t)k);
    *L = complement(fr);
    *R = complement(fl);
  }
  return 1;
}

/* ---- record buffer ----------------------------------------------------- */

typedef struct {
  uint8_t *buf;
  int64_t n, cap;
  size_t stride; /* k letters + left + right */
} recbuf;

static int recbuf_push(recbuf *b, const uint8_t *key, size_t k, uint8_t L,
                       uint8_t R) {
  if (b->n == b->cap) {
    int64_t nc = b->cap ? b->cap * 2 : 1024;
    uint8_t *nb = (uint8_t *)realloc(b->buf, (size_t)nc * b->stride);
    if (!nb) return -1;
    b->buf = nb;
    b->cap = nc;
  }
  uint8_t *r = b->buf + (size_t)b->n * b->stride;
  memcpy(r, key, k);
  r[k] = L;
  r[k + 1] = R;
  b->n++;
  return 0;
}

static int cmp_key(const void *a, const void *b, void *arg) {
  return memcmp(a, b, *(const size_t *)arg);
}

/* ---- packing for export ------------------------------------------------ */

/* k-mer value N = sum_j code(s_j) * 4^(k-1-j); W 64-bit words, most
 * significant first (the last word holds the low 64 bits). */
static void pack_key(const uint8_t *key, uint32_t k, uint32_t W,
                     uint64_t *out) {
  memset(out, 0, sizeof(uint64_t) * W);
  for (uint32_t j = 0; j < k; j++) {
    uint32_t bit = 2 * (k - 1 - j);
    out[W - 1 - bit / 64] |= (uint64_t)letter_index(key[j]) << (bit % 64);
  }
}

static void unpack_key(const uint64_t *words, uint32_t k, uint32_t W,
                       uint8_t *key) {
  static const uint8_t letters[4] = {'A', 'C', 'G', 'T'};
  for (uint32_t j = 0; j < k; j++) {
    uint32_t bit = 2 * (k - 1 - j);
    key[j] = letters[(words[W - 1 - bit / 64] >> (bit % 64)) & 3];
  }
}

static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

uint64_t oracle_shard_of(const uint64_t *key, uint32_t W, uint64_t S) {
  uint64_t h = 0;
  for (uint32_t i = 0; i < W; i++) h = mix64(h ^ key[i]);
  return h % S;
}

/* ---- classification ---------------------------------------------------- */

/* Section II-C: a k-mer of depth d is extended only if no more than
 * t_hq = max(t_base, e * d) observations contradict its most common
 * extension; otherwise it is a fork.  Section II-B: an extension must be
 * seen often enough to count at all; fewer than t_min_ext observations of
 * the most common base make the side a dead end.  Readings: the letters F
 * (fork) and X (dead end) name the two non-unique outcomes; a tie for the
 * most common base is a fork; e is err_ppm / 10^6 and the comparison is
 * done in integers scaled by 10^6 so that it is exact. */
uint8_t oracle_classify_side(const uint64_t c[4], uint64_t depth,
                             const oracle_params *p) {
  static const uint8_t letters[4] = {'A', 'C', 'G', 'T'};
  uint64_t m = 0, sum = 0;
  int best = 0;
  for (int b = 0; b < 4; b++) {
    sum += c[b];
    if (c[b] > m) {
      m = c[b];
      best = b;
    }
  }
  if (m < p->t_min_ext) return 'X';
  int n_at_max = 0;
  for (int b = 0; b < 4; b++) n_at_max += (c[b] == m);
  if (n_at_max >= 2) return 'F';
  uint64_t alt = sum - m;
  uint64_t floor_ = (uint64_t)p->t_base * 1000000ULL;
  uint64_t slope = (uint64_t)p->err_ppm * depth;
  uint64_t t_hq = floor_ > slope ? floor_ : slope;
  return alt * 1000000ULL <= t_hq ? letters[best] : 'F';
}

/* ---- grouping ---------------------------------------------------------- */

static int check_params(const oracle_params *p) {
  if (!p || p->k < 1 || p->k > 127 || p->min_count < 1) return -1;
  return 0;
}

/* Sort the records, sum equal keys, apply the threshold and export. */
static int group_records(recbuf *b, const oracle_params *p, oracle_table **out) {
  size_t k = p->k;
  const uint32_t W = (p->k + 31) / 32;
  if (b->n > 1) qsort_r(b->buf, (size_t)b->n, b->stride, cmp_key, &k);

  oracle_table *t = (oracle_table *)calloc(1, sizeof(oracle_table));
  if (!t) return -1;
  t->k = p->k;
  t->W = W;
  /* first pass: distinct keys and kept rows */
  int64_t kept = 0;
  for (int64_t i = 0; i < b->n;) {
    const uint8_t *ki = b->buf + (size_t)i * b->stride;
    int64_t j = i + 1;
    while (j < b->n && memcmp(ki, b->buf + (size_t)j * b->stride, k) == 0) j++;
    t->n_distinct++;
    if ((uint64_t)(j - i) >= p->min_count) kept++;
    i = j;
  }
  t->keys = (uint64_t *)malloc(sizeof(uint64_t) * W * (size_t)(kept ? kept : 1));
  t->counts = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(kept ? kept : 1));
  t->ext = (uint32_t *)malloc(sizeof(uint32_t) * 8 * (size_t)(kept ? kept : 1));
  t->codes = (uint8_t *)malloc(2 * (size_t)(kept ? kept : 1));
  if (!t->keys || !t->counts || !t->ext || !t->codes) {
    oracle_free(t);
    return -1;
  }
  int64_t row = 0;
  for (int64_t i = 0; i < b->n;) {
    const uint8_t *ki = b->buf + (size_t)i * b->stride;
    uint64_t count = 0, left[4] = {0, 0, 0, 0}, right[4] = {0, 0, 0, 0};
    int64_t j = i;
    while (j < b->n && memcmp(ki, b->buf + (size_t)j * b->stride, k) == 0) {
      const uint8_t *r = b->buf + (size_t)j * b->stride;
      count++;
      if (r[k]) left[letter_index(r[k])]++;
      if (r[k + 1]) right[letter_index(r[k + 1])]++;
      j++;
    }
    t->n_windows += count;
    for (int c = 0; c < 4; c++) {
      t->sum_left += left[c];
      t->sum_right += right[c];
    }
    if (count >= p->min_count) {
      if (count > 0xffffffffULL) {
        oracle_free(t);
        return -2;
      }
      pack_key(ki, p->k, W, t->keys + (size_t)row * W);
      t->counts[row] = (uint32_t)count;
      for (int c = 0; c < 4; c++) {
        t->ext[row * 8 + c] = (uint32_t)left[c];
        t->ext[row * 8 + 4 + c] = (uint32_t)right[c];
      }
      t->codes[row * 2] = oracle_classify_side(left, count, p);
      t->codes[row * 2 + 1] = oracle_classify_side(right, count, p);
      row++;
    }
    i = j;
  }
  t->n_rows = row;
  *out = t;
  return 0;
}

/* ---- entry points ------------------------------------------------------ */

/* Collect the records of reads [r0, r1) into b; keep only shard s of S when
 * S > 0. */
static int collect(const uint8_t *seq, const uint8_t *qual,
                   const int64_t *offsets, int64_t r0, int64_t r1,
                   const oracle_params *p, uint64_t S, uint64_t s, recbuf *b) {
  const size_t k = p->k;
  const uint32_t W = (p->k + 31) / 32;
  uint8_t *fwd = (uint8_t *)malloc(k), *rc = (uint8_t *)malloc(k);
  uint8_t *key = (uint8_t *)malloc(k);
  uint64_t words[4];
  int rc_ = (fwd && rc && key) ? 0 : -1;
  for (int64_t r = r0; r < r1 && rc_ == 0; r++) {
    const uint8_t *sr = seq + offsets[r];
    const uint8_t *qr = qual + offsets[r];
    const int64_t len = offsets[r + 1] - offsets[r];
    for (int64_t i = 0; i + (int64_t)k <= len; i++) {
      uint8_t L, R;
      if (!window_record(sr, qr, len, i, p, fwd, rc, key, &L, &R)) continue;
      if (S > 0) {
        pack_key(key, p->k, W, words);
        if (oracle_shard_of(words, W, S) != s) continue;
      }
      if (recbuf_push(b, key, k, L, R)) {
        rc_ = -1;
        break;
      }
    }
  }
  free(fwd);
  free(rc);
  free(key);
  return rc_;
}

static int check_reads(const int64_t *offsets, int64_t n_reads) {
  if (n_reads < 0 || (n_reads > 0 && !offsets)) return -1;
  for (int64_t r = 0; r < n_reads; r++)
    if (offsets[r + 1] < offsets[r]) return -1;
  return 0;
}

int oracle_count(const uint8_t *seq, const uint8_t *qual,
                 const int64_t *offsets, int64_t n_reads,
                 const oracle_params *p, oracle_table **out) {
  if (!out || check_params(p) || check_reads(offsets, n_reads)) return -1;
  recbuf b = {NULL, 0, 0, (size_t)p->k + 2};
  int rc = collect(seq, qual, offsets, 0, n_reads, p, 0, 0, &b);
  if (rc == 0) rc = group_records(&b, p, out);
  free(b.buf);
  return rc;
}

int oracle_count_shard(const uint8_t *seq, const uint8_t *qual,
                       const int64_t *offsets, int64_t n_reads,
                       const oracle_params *p, uint64_t S, uint64_t s,
                       oracle_table **out) {
  if (!out || check_params(p) || check_reads(offsets, n_reads) || S == 0 ||
      s >= S)
    return -1;
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  recbuf *parts = (recbuf *)calloc((size_t)nt, sizeof(recbuf));
  if (!parts) return -1;
  int err = 0;
#pragma omp parallel num_threads(nt)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    parts[t].stride = (size_t)p->k + 2;
    int64_t r0 = n_reads * t / nt, r1 = n_reads * (t + 1) / nt;
    if (collect(seq, qual, offsets, r0, r1, p, S, s, &parts[t])) {
#pragma omp atomic write
      err = 1;
    }
  }
  recbuf all = {NULL, 0, 0, (size_t)p->k + 2};
  for (int t = 0; t < nt && !err; t++) {
    for (int64_t i = 0; i < parts[t].n; i++) {
      const uint8_t *r = parts[t].buf + (size_t)i * all.stride;
      if (recbuf_push(&all, r, p->k, r[p->k], r[p->k + 1])) {
        err = 1;
        break;
      }
    }
  }
  for (int t = 0; t < nt; t++) free(parts[t].buf);
  free(parts);
  int rc = err ? -1 : group_records(&all, p, out);
  free(all.buf);
  return rc;
}

typedef struct {
  const uint8_t *letters; /* k letters */
  int64_t index;
} query;

static size_t g_qk; /* key length for the query comparator (set per call) */

static int cmp_query(const void *a, const void *b) {
  return memcmp(((const query *)a)->letters, ((const query *)b)->letters, g_qk);
}

int oracle_count_keys(const uint8_t *seq, const uint8_t *qual,
                      const int64_t *offsets, int64_t n_reads,
                      const oracle_params *p, const uint64_t *qkeys,
                      int64_t nq, uint64_t *counts, uint64_t *ext) {
  if (check_params(p) || check_reads(offsets, n_reads) || nq < 0 ||
      (nq > 0 && (!qkeys || !counts || !ext)))
    return -1;
  const size_t k = p->k;
  const uint32_t W = (p->k + 31) / 32;
  memset(counts, 0, sizeof(uint64_t) * (size_t)nq);
  memset(ext, 0, sizeof(uint64_t) * 8 * (size_t)nq);
  if (nq == 0) return 0;
  uint8_t *text = (uint8_t *)malloc(k * (size_t)nq);
  query *qs = (query *)malloc(sizeof(query) * (size_t)nq);
  if (!text || !qs) {
    free(text);
    free(qs);
    return -1;
  }
  for (int64_t i = 0; i < nq; i++) {
    unpack_key(qkeys + (size_t)i * W, p->k, W, text + (size_t)i * k);
    qs[i].letters = text + (size_t)i * k;
    qs[i].index = i;
  }
  g_qk = k;
  qsort(qs, (size_t)nq, sizeof(query), cmp_query);
  int err = 0;
#pragma omp parallel
  {
    uint64_t *lc = (uint64_t *)calloc((size_t)nq * 9, sizeof(uint64_t));
    uint8_t *fwd = (uint8_t *)malloc(k), *rc = (uint8_t *)malloc(k);
    uint8_t *key = (uint8_t *)malloc(k);
    if (!lc || !fwd || !rc || !key) {
#pragma omp atomic write
      err = 1;
    } else {
#pragma omp for schedule(dynamic, 4096)
      for (int64_t r = 0; r < n_reads; r++) {
        const uint8_t *sr = seq + offsets[r];
        const uint8_t *qr = qual + offsets[r];
        const int64_t len = offsets[r + 1] - offsets[r];
        for (int64_t i = 0; i + (int64_t)k <= len; i++) {
          uint8_t L, R;
          if (!window_record(sr, qr, len, i, p, fwd, rc, key, &L, &R)) continue;
          query probe = {key, 0};
          const query *hit = (const query *)bsearch(&probe, qs, (size_t)nq,
                                                    sizeof(query), cmp_query);
          if (!hit) continue;
          uint64_t *acc = lc + (size_t)hit->index * 9;
          acc[0]++;
          if (L) acc[1 + letter_index(L)]++;
          if (R) acc[5 + letter_index(R)]++;
        }
      }
#pragma omp critical
      for (int64_t i = 0; i < nq; i++) {
        counts[i] += lc[i * 9];
        for (int c = 0; c < 8; c++) ext[i * 8 + c] += lc[i * 9 + 1 + c];
      }
    }
    free(lc);
    free(fwd);
    free(rc);
    free(key);
  }
  free(text);
  free(qs);
  return err ? -1 : 0;
}

/* OpenMP threads of the calling thread's later parallel regions (a caller
 * that runs several shard counts at once gives each one thread).  Touches
 * no result. */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

void oracle_free(oracle_table *t) {
  if (!t) return;
  free(t->keys);
  free(t->counts);
  free(t->ext);
  free(t->codes);
  free(t);
}
