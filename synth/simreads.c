/*
 * Seeded synthetic genomes and short reads.
 *
 * This module produces test and benchmark INPUTS only.  It holds none of the
 * k-mer analysis arithmetic: it draws random genomes, samples fragments from
 * them, applies substitution errors and draws Phred qualities.  Both the CPU
 * oracle and the GPU library consume its output; neither is used here.
 *
 * Randomness is counter based: every draw is mix64(key + (ctr + 1) * phi),
 * where mix64 is the SplitMix64 output function (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) and phi is
 * the 64-bit golden-ratio increment.  A draw therefore depends only on
 * (seed, stream, counter), so the output is identical for any thread count.
 *
 * The read model follows the MGSim / WGSim description used by the paper
 * (Section III-A): genomes are sampled with probability proportional to
 * abundance x length, fragments start uniformly, strand is 50/50, and every
 * base is independently substituted with probability p_err.
 */
#include <stdint.h>
#include <string.h>

#define PHI 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed ^ mix64(stream * PHI + 0x5851f42d4c957f2dULL));
}

static inline uint64_t draw(uint64_t key, uint64_t ctr) {
  return mix64(key + (ctr + 1) * PHI);
}

/* Uniform integer in [0, n) from the high 63 bits of a draw (n > 0). */
static inline uint64_t below(uint64_t d, uint64_t n) {
  return (uint64_t)(((unsigned __int128)(d >> 1) * n) >> 63);
}

static inline uint8_t comp_ascii(uint8_t c) {
  switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    default: return 'N';
  }
}

/* Smallest index i with u < cdf[i]; cdf is non-decreasing, cdf[n-1] > any u. */
static inline int cdf_pick(const uint64_t *cdf, int n, uint64_t u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (u < cdf[mid]) hi = mid; else lo = mid + 1;
  }
  return lo;
}

/*
 * Genome of `len` iid bases: P(C) = P(G) = gc/2, P(A) = P(T) = (1-gc)/2, with
 * gc = gc_thresh / 2^32.  Written as ASCII into out[0..len).
 */
void sim_genome(uint64_t seed, uint64_t stream, int64_t len, uint64_t gc_thresh,
                uint8_t *out) {
  const uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < len; i++) {
    uint64_t d = draw(key, (uint64_t)i);
    uint64_t u = d >> 32;
    int bit = (int)(d & 1);
    if (u < gc_thresh) out[i] = bit ? 'G' : 'C';
    else out[i] = bit ? 'T' : 'A';
  }
}

/*
 * Per-fragment layout: genome index, start, strand, insert size and the two
 * read lengths.  Lengths are drawn uniformly in [len_min, len_max]; insert
 * sizes from the tabulated distribution ins_cdf over [ins_min, ins_min+ins_n),
 * raised to at least the longer mate and lowered to the genome length.
 *
 *   cum_w[g]   cumulative genome weights scaled to 2^63 (non-decreasing,
 *              cum_w[n_genomes-1] = 2^63)
 *   paired     0: one read per fragment (insert = read length); 1: two reads
 * Outputs (per fragment f): frag_g, frag_pos, frag_strand, frag_ins, and
 * read_len[f * (1 + paired) + m].
 */
void sim_layout(uint64_t seed, int64_t n_frag, int paired,
                const int64_t *genome_len, int n_genomes, const uint64_t *cum_w,
                int len_min, int len_max, const uint64_t *ins_cdf, int ins_min,
                int ins_n, int32_t *frag_g, int64_t *frag_pos,
                uint8_t *frag_strand, int32_t *frag_ins, int32_t *read_len) {
  const uint64_t key = stream_key(seed, 1);
  const int nm = paired ? 2 : 1;
#pragma omp parallel for schedule(static)
  for (int64_t f = 0; f < n_frag; f++) {
    uint64_t d0 = draw(key, (uint64_t)f * 8 + 0);
    uint64_t d1 = draw(key, (uint64_t)f * 8 + 1);
    uint64_t d2 = draw(key, (uint64_t)f * 8 + 2);
    int g = cdf_pick(cum_w, n_genomes, d0 >> 1);
    int64_t glen = genome_len[g];
    int lmax = 0;
    for (int m = 0; m < nm; m++) {
      uint64_t dl = draw(key, (uint64_t)f * 8 + 3 + m);
      int l = len_min + (int)below(dl, (uint64_t)(len_max - len_min + 1));
      if (l > glen) l = (int)glen;
      read_len[f * nm + m] = l;
      if (l > lmax) lmax = l;
    }
    int ins;
    if (paired) {
      ins = ins_min + cdf_pick(ins_cdf, ins_n, d2 >> 32);
      if (ins < lmax) ins = lmax;
    } else {
      ins = lmax;
    }
    if (ins > glen) ins = (int)glen;
    frag_g[f] = g;
    frag_ins[f] = ins;
    frag_strand[f] = (uint8_t)(d1 >> 63);
    frag_pos[f] = (int64_t)below(d1, (uint64_t)(glen - ins + 1));
  }
}

/*
 * Fill reads.  Read r = f * (1 + paired) + m starts at offsets[r].
 * Mate 0 is the first read_len bases of the oriented fragment; mate 1 is the
 * reverse complement of its last read_len bases.  Each base is substituted
 * with probability err_thresh / 2^32 (to one of the three other bases,
 * uniformly); its quality comes from q_ok_cdf or, for a substituted base,
 * q_err_cdf (tables over Phred 0..n_q-1), written as Phred + 33.  A base
 * becomes 'N' with probability n_thresh / 2^32.
 */
void sim_fill(uint64_t seed, int64_t n_frag, int paired, const uint8_t *genomes,
              const int64_t *genome_off, const int32_t *frag_g,
              const int64_t *frag_pos, const uint8_t *frag_strand,
              const int32_t *frag_ins, const int32_t *read_len,
              const int64_t *offsets, uint64_t err_thresh,
              const uint64_t *q_ok_cdf, const uint64_t *q_err_cdf, int n_q,
              uint64_t n_thresh, uint8_t *seq, uint8_t *qual) {
  const uint64_t ekey = stream_key(seed, 2);
  const uint64_t qkey = stream_key(seed, 3);
  const int nm = paired ? 2 : 1;
  static const uint8_t other[4][3] = {
      {'C', 'G', 'T'}, {'A', 'G', 'T'}, {'A', 'C', 'T'}, {'A', 'C', 'G'}};
#pragma omp parallel for schedule(static)
  for (int64_t f = 0; f < n_frag; f++) {
    const uint8_t *g = genomes + genome_off[frag_g[f]];
    const int64_t pos = frag_pos[f];
    const int ins = frag_ins[f];
    const int strand = frag_strand[f];
    for (int m = 0; m < nm; m++) {
      const int64_t r = f * nm + m;
      const int L = read_len[r];
      uint8_t *s = seq + offsets[r];
      uint8_t *q = qual + offsets[r];
      for (int j = 0; j < L; j++) {
        uint8_t b;
        /* oriented fragment x: strand ? comp(g[pos+ins-1-x]) : g[pos+x] */
        if (m == 0) {
          b = strand ? comp_ascii(g[pos + ins - 1 - j]) : g[pos + j];
        } else {
          b = strand ? g[pos + j] : comp_ascii(g[pos + ins - 1 - j]);
        }
        const uint64_t ctr = (uint64_t)offsets[r] + (uint64_t)j;
        const uint64_t de = draw(ekey, ctr);
        const uint64_t dq = draw(qkey, ctr);
        int err = (de >> 32) < err_thresh;
        if (err) {
          int bi = b == 'A' ? 0 : b == 'C' ? 1 : b == 'G' ? 2 : 3;
          b = other[bi][(de & 0xffffffffULL) % 3];
        }
        int ph = cdf_pick(err ? q_err_cdf : q_ok_cdf, n_q, dq >> 32);
        if ((dq & 0xffffffffULL) < n_thresh) b = 'N';
        s[j] = b;
        q[j] = (uint8_t)(ph + 33);
      }
    }
  }
}
