/*
 * CPU oracle for iterative graph pruning -- TEST INFRASTRUCTURE ONLY.
 *
 * What it computes (paper Section II, the iterative graph pruning subsection
 * and its Algorithm 2, after IDBA-UD): a threshold tau starts at 1 and grows
 * by the factor (1 + alpha) after every sweep while it stays below the
 * largest depth of the remaining contigs; a sweep removes every contig of at
 * most 2k bases whose depth is at most min(tau, beta * the depth of its
 * neighbourhood).
 *
 * Readings (the paper leaves these open):
 *  P1 depth(c) is the mean count of c's k-mers: the sum of their counts
 *     divided by their number.
 *  P2 The neighbourhood's depth is the pooled mean over the neighbouring
 *     contigs still present: the sum of their k-mers' counts divided by the
 *     number of their k-mers.  A contig with no neighbour left is kept.
 *  P3 Contig c' neighbours c when c' (c' != c) holds a k-mer that overlaps
 *     c's first k-mer by k-1 bases on its left (b + S[0..k-1)) or c's last
 *     k-mer by k-1 bases on its right (S[1..k) + b), for any base b, in
 *     either orientation: the (k-1)-overlap adjacency of the graph's
 *     vertices at the contig's ends, whatever the extension codes say.
 *     Each neighbour counts once.
 *  P4 Sweeps are synchronous: every decision of a sweep sees the contigs as
 *     they were when it started; its removals take effect at its end (the
 *     parallel form updates the neighbourhoods after each iteration).
 *  P5 The loop runs while tau < the largest depth of the remaining contigs,
 *     that maximum taken again after every sweep (Algorithm 2's condition).
 *     The early stop on a sweep that removes nothing is not applied: at
 *     tau = 1 nothing of depth >= 1 can go, so it would end every run there.
 *  P6 length(c) is the number of bases, k + n_kmers - 1; "<= 2k" inclusive.
 *  P7 Arithmetic in IEEE double, one rounding per operation, in this order:
 *     d = sum / n; nd = sum_nb / n_nb; cut = min(tau, beta * nd); remove iff
 *     d <= cut; tau_next = tau * g with g = 1 + alpha rounded once.
 *
 * Pins: the Python tests check this oracle against an independent brute
 * force (dictionaries over k-mer strings) on random tables, against closed
 * forms (a low-depth tip or bubble branch next to a deep genome is removed
 * at the first sweep whose tau reaches its depth, the genome side never),
 * and against invariants (contigs longer than 2k and contigs without
 * neighbours stay; beta = 0 removes nothing of positive depth; the number of
 * sweeps is the number of tau values below the running maximum depth).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int pr_is_acgt(char c) { return c == 'A' || c == 'C' || c == 'G' || c == 'T'; }
static char pr_comp(char c) {
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
} kref;

static uint32_t pr_k;
static int cmp_kref(const void *a, const void *b) {
  return memcmp(((const kref *)a)->key, ((const kref *)b)->key, pr_k);
}

/* canonical form of w (k letters) into out */
static void canonical(const char *w, uint32_t k, char *rc, char *out) {
  for (uint32_t j = 0; j < k; j++) rc[j] = pr_comp(w[k - 1 - j]);
  memcpy(out, memcmp(rc, w, k) < 0 ? rc : w, k);
}

/* contig holding the k-mer w (either orientation), or -1 */
static int64_t holder(const kref *refs, int64_t nref, const char *w, uint32_t k, char *rc,
                      char *canon) {
  canonical(w, k, rc, canon);
  int64_t lo = 0, hi = nref;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (memcmp(refs[mid].key, canon, k) < 0) lo = mid + 1; else hi = mid;
  }
  return (lo < nref && memcmp(refs[lo].key, canon, k) == 0) ? refs[lo].contig : -1;
}

int oracle_prune(const char *cseq, const int64_t *coff, const uint64_t *depth,
                 int64_t n_contigs, uint32_t k, double alpha, double beta,
                 int32_t *removed_at, int64_t *sweeps) {
  if (k < 1 || k > 127 || n_contigs < 0 || !removed_at || !sweeps ||
      (n_contigs > 0 && (!cseq || !coff || !depth)) || !(alpha >= 1e-3 && alpha <= 1e3) ||
      !(beta >= 0.0 && beta <= 1e6))
    return -1;
  *sweeps = 0;
  int64_t nref = 0;
  for (int64_t c = 0; c < n_contigs; c++) {
    const int64_t len = coff[c + 1] - coff[c];
    if (len < (int64_t)k) return -1; /* a contig holds at least one k-mer */
    for (int64_t p = coff[c]; p < coff[c + 1]; p++)
      if (!pr_is_acgt(cseq[p])) return -1;
    nref += len - k + 1;
  }
  int rcode = -1;
  kref *refs = (kref *)malloc(sizeof(kref) * (size_t)(nref > 0 ? nref : 1));
  char *store = (char *)malloc((size_t)(nref > 0 ? nref : 1) * k);
  int64_t *nb = (int64_t *)malloc(sizeof(int64_t) * 8 * (size_t)(n_contigs > 0 ? n_contigs : 1));
  int *nnb = (int *)calloc((size_t)(n_contigs > 0 ? n_contigs : 1), sizeof(int));
  char *alive = (char *)malloc((size_t)(n_contigs > 0 ? n_contigs : 1));
  char *go = (char *)malloc((size_t)(n_contigs > 0 ? n_contigs : 1));
  char *w = (char *)malloc(k), *rc = (char *)malloc(k), *canon = (char *)malloc(k);
  if (!refs || !store || !nb || !nnb || !alive || !go || !w || !rc || !canon) goto done;
  /* ---- every contig k-mer, canonical, with its contig */
  {
    int64_t m = 0;
    for (int64_t c = 0; c < n_contigs; c++)
      for (int64_t p = coff[c]; p + (int64_t)k <= coff[c + 1]; p++) {
        char *key = store + (size_t)m * k;
        canonical(cseq + p, k, rc, key);
        refs[m].key = key;
        refs[m].contig = c;
        m++;
      }
    pr_k = k;
    qsort(refs, (size_t)nref, sizeof(kref), cmp_kref);
    for (int64_t i = 1; i < nref; i++) /* the contigs must not share a k-mer */
      if (memcmp(refs[i - 1].key, refs[i].key, k) == 0) goto done;
  }
  /* ---- neighbours (P3) */
  for (int64_t c = 0; c < n_contigs; c++) {
    const char *s = cseq + coff[c];
    const int64_t len = coff[c + 1] - coff[c];
    for (int side = 0; side < 2; side++)
      for (int b = 0; b < 4; b++) {
        if (side == 0) { /* b + first k-mer's first k-1 bases */
          w[0] = "ACGT"[b];
          memcpy(w + 1, s, k - 1);
        } else { /* last k-mer's last k-1 bases + b */
          memcpy(w, s + len - (k - 1), k - 1);
          w[k - 1] = "ACGT"[b];
        }
        const int64_t j = holder(refs, nref, w, k, rc, canon);
        if (j < 0 || j == c) continue;
        int seen = 0;
        for (int x = 0; x < nnb[c]; x++) seen = seen || nb[8 * c + x] == j;
        if (!seen) nb[8 * c + nnb[c]++] = j;
      }
  }
  /* ---- Algorithm 2 */
  for (int64_t c = 0; c < n_contigs; c++) {
    alive[c] = 1;
    removed_at[c] = -1;
  }
  {
    const double g = 1.0 + alpha;
    double tau = 1.0;
    for (int64_t sweep = 0;; sweep++) {
      double mx = 0.0; /* largest depth of the remaining contigs (P5) */
      int any = 0;
      for (int64_t c = 0; c < n_contigs; c++)
        if (alive[c]) {
          const double d = (double)depth[c] / (double)(coff[c + 1] - coff[c] - k + 1);
          if (!any || d > mx) mx = d;
          any = 1;
        }
      if (!any || !(tau < mx)) break;
      for (int64_t c = 0; c < n_contigs; c++) {
        go[c] = 0;
        const int64_t len = coff[c + 1] - coff[c];
        if (!alive[c] || len > 2 * (int64_t)k) continue; /* P6 */
        uint64_t sum_nb = 0, n_nb = 0;
        for (int x = 0; x < nnb[c]; x++) {
          const int64_t j = nb[8 * c + x];
          if (!alive[j]) continue;
          sum_nb += depth[j];
          n_nb += (uint64_t)(coff[j + 1] - coff[j] - k + 1);
        }
        if (n_nb == 0) continue; /* P2: no neighbour left */
        const double d = (double)depth[c] / (double)(len - k + 1);
        const double nd = (double)sum_nb / (double)n_nb;
        const double bnd = beta * nd;
        const double cut = tau < bnd ? tau : bnd;
        go[c] = d <= cut;
      }
      for (int64_t c = 0; c < n_contigs; c++) /* P4: applied after the sweep */
        if (go[c]) {
          alive[c] = 0;
          removed_at[c] = (int32_t)sweep;
        }
      *sweeps = sweep + 1;
      tau = tau * g;
    }
  }
  rcode = 0;
done:
  free(refs);
  free(store);
  free(nb);
  free(nnb);
  free(alive);
  free(go);
  free(w);
  free(rc);
  free(canon);
  return rcode;
}
