"""Seeded synthetic metagenome reads for tests and benchmarks.

This package produces inputs only.  It contains none of the k-mer analysis
arithmetic (no windows, canonical forms, hashing, counting or classification):
both the CPU oracle and the GPU library consume what it writes, and it imports
neither of them.

The read model mirrors the synthetic data the paper uses for its weak-scaling
study (Section III-A, MGSim): genomes are random, their relative abundances are
drawn from a log-normal distribution, fragments are sampled in proportion to
abundance x genome length, reads come from both strands and carry iid
substitution errors.  Qualities are Phred+33: clip(rint(N(35, 5)), 2, 41) for a
correct base and clip(rint(N(15, 5)), 2, 41) for a substituted one.

The per-base work runs in a small C library (``simreads.c``, OpenMP) with a
counter-based generator, so results do not depend on the thread count.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "simreads.c")
_SO = os.path.join(_HERE, "libsimreads.so")
_lib = None

BASE_SEED = 1809_07014


def build(force: bool = True) -> str:
    """Compile the C core into ``libsimreads.so`` next to this file."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, u64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
        lib.sim_genome.argtypes = [u64, u64, i64, u64, P]
        lib.sim_genome.restype = None
        lib.sim_layout.argtypes = [u64, i64, i32, P, i32, P, i32, i32, P, i32,
                                   i32, P, P, P, P, P]
        lib.sim_layout.restype = None
        lib.sim_fill.argtypes = [u64, i64, i32, P, P, P, P, P, P, P, P, u64, P,
                                 P, i32, u64, P, P]
        lib.sim_fill.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _norm_cdf(x: float) -> float:
    return 0.5 * (1.0 + math.erf(x / math.sqrt(2.0)))


def phred_cdf(mean: float, sd: float, lo: int = 2, hi: int = 41) -> np.ndarray:
    """CDF table (scaled to 2^32) of clip(rint(N(mean, sd)), lo, hi) over 0..hi."""
    cdf = np.zeros(hi + 1, dtype=np.uint64)
    for q in range(hi + 1):
        if q < lo:
            p = 0.0
        elif q >= hi:
            p = 1.0
        else:
            p = _norm_cdf((q + 0.5 - mean) / sd)
        cdf[q] = min(int(round(p * 2.0**32)), 2**32)
    cdf[hi] = 2**32
    return cdf


def insert_cdf(mean: float, sd: float, lo: int, hi: int) -> np.ndarray:
    """CDF table (scaled to 2^32) of clip(rint(N(mean, sd)), lo, hi) over lo..hi."""
    n = hi - lo + 1
    cdf = np.zeros(n, dtype=np.uint64)
    for i in range(n):
        v = lo + i
        p = 1.0 if v >= hi else _norm_cdf((v + 0.5 - mean) / sd)
        cdf[i] = min(int(round(p * 2.0**32)), 2**32)
    cdf[n - 1] = 2**32
    return cdf


@dataclass
class Reads:
    """Concatenated ASCII reads: read r is seq[offsets[r]:offsets[r+1]]."""
    seq: np.ndarray          # uint8, ASCII bases
    qual: np.ndarray         # uint8, Phred + 33
    offsets: np.ndarray      # int64, n_reads + 1, offsets[0] == 0
    meta: dict = field(default_factory=dict)

    @property
    def n_reads(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_bases(self) -> int:
        return int(self.offsets[-1])

    def slice(self, r0: int, r1: int) -> "Reads":
        a, b = int(self.offsets[r0]), int(self.offsets[r1])
        return Reads(self.seq[a:b], self.qual[a:b],
                     (self.offsets[r0:r1 + 1] - a).astype(np.int64),
                     dict(self.meta, slice=(r0, r1)))

    def strings(self):
        """(sequence, quality) pairs as Python strings (small inputs only)."""
        out = []
        for r in range(self.n_reads):
            a, b = int(self.offsets[r]), int(self.offsets[r + 1])
            out.append((self.seq[a:b].tobytes().decode(),
                        self.qual[a:b].tobytes().decode()))
        return out

    @staticmethod
    def from_strings(pairs) -> "Reads":
        seqs = [s.encode() for s, _ in pairs]
        quals = [q.encode() for _, q in pairs]
        for s, q in zip(seqs, quals):
            if len(s) != len(q):
                raise ValueError("sequence and quality lengths differ")
        lens = np.array([len(s) for s in seqs], dtype=np.int64)
        offsets = np.zeros(len(seqs) + 1, dtype=np.int64)
        np.cumsum(lens, out=offsets[1:])
        seq = np.frombuffer(b"".join(seqs), dtype=np.uint8).copy()
        qual = np.frombuffer(b"".join(quals), dtype=np.uint8).copy()
        return Reads(seq, qual, offsets)


def genomes(seed: int, lengths, gcs) -> tuple[np.ndarray, np.ndarray]:
    """Random genomes, concatenated.  Returns (ascii, offsets[n+1])."""
    lib = _load()
    lengths = np.asarray(lengths, dtype=np.int64)
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    out = np.empty(int(off[-1]), dtype=np.uint8)
    for g, (L, gc) in enumerate(zip(lengths, gcs)):
        view = out[off[g]:off[g + 1]]
        lib.sim_genome(seed, 1000 + g, int(L), int(round(gc * 2.0**32)),
                       _ptr(view))
    return out, off


def simulate(seed: int, genome_ascii: np.ndarray, genome_off: np.ndarray,
             abundance, n_frag: int, paired: bool, len_min: int = 150,
             len_max: int = 150, p_err: float = 0.005, n_rate: float = 0.0,
             ins_mean: float = 300.0, ins_sd: float = 30.0,
             q_ok=(35.0, 5.0), q_err=(15.0, 5.0)) -> Reads:
    """Sample reads from the given genomes (see module docstring)."""
    lib = _load()
    glen = np.diff(genome_off).astype(np.int64)
    ng = len(glen)
    w = np.asarray(abundance, dtype=np.float64) * glen
    cum = np.cumsum(w) / w.sum()
    cum_w = np.minimum(np.round(cum * 2.0**63), 2.0**63).astype(np.uint64)
    cum_w[-1] = np.uint64(2**63)
    ins_lo, ins_hi = max(len_max, 1), max(len_max, int(ins_mean + 10 * ins_sd))
    icdf = insert_cdf(ins_mean, ins_sd, ins_lo, ins_hi)
    nm = 2 if paired else 1
    fg = np.empty(n_frag, np.int32)
    fp = np.empty(n_frag, np.int64)
    fs = np.empty(n_frag, np.uint8)
    fi = np.empty(n_frag, np.int32)
    rl = np.empty(n_frag * nm, np.int32)
    lib.sim_layout(seed, n_frag, int(paired), _ptr(glen), ng, _ptr(cum_w),
                   len_min, len_max, _ptr(icdf), ins_lo, len(icdf), _ptr(fg),
                   _ptr(fp), _ptr(fs), _ptr(fi), _ptr(rl))
    offsets = np.zeros(n_frag * nm + 1, dtype=np.int64)
    np.cumsum(rl, out=offsets[1:])
    n = int(offsets[-1])
    seq = np.empty(n, np.uint8)
    qual = np.empty(n, np.uint8)
    qok = phred_cdf(*q_ok)
    qer = phred_cdf(*q_err)
    lib.sim_fill(seed, n_frag, int(paired), _ptr(genome_ascii),
                 _ptr(genome_off), _ptr(fg), _ptr(fp), _ptr(fs), _ptr(fi),
                 _ptr(rl), _ptr(offsets), int(round(p_err * 2.0**32)),
                 _ptr(qok), _ptr(qer), len(qok), int(round(n_rate * 2.0**32)),
                 _ptr(seq), _ptr(qual))
    meta = dict(seed=seed, n_genomes=ng, genome_bases=int(genome_off[-1]),
                paired=paired, p_err=p_err, n_rate=n_rate)
    return Reads(seq, qual, offsets, meta)


def metagenome(seed: int, n_genomes: int, len_lo: int, len_hi: int,
               gc_lo: float, gc_hi: float, sigma: float):
    """Genome lengths ~ U{len_lo..len_hi}, GC ~ U(gc_lo, gc_hi) and
    abundances ~ exp(N(0, sigma)), drawn with numpy's PCG64 from ``seed``."""
    rng = np.random.default_rng(seed)
    lengths = rng.integers(len_lo, len_hi + 1, size=n_genomes)
    gcs = rng.uniform(gc_lo, gc_hi, size=n_genomes)
    ab = np.exp(rng.normal(0.0, sigma, size=n_genomes))
    return lengths.astype(np.int64), gcs, ab


def config(i: int, scale: float = 1.0, seed_offset: int = 0) -> Reads:
    """Reads of workload ``i`` (1-based, see below), optionally scaled down.

    1  one 50 kbp genome (GC 0.5), 6,667 single-end 150 bp reads (20x),
       0.5 % substitutions -- the small k = 21 case.
    2  100 genomes of 2-5 Mbp, GC ~ U(0.3, 0.7), abundance log-normal(0, 1.5),
       10M paired 150 bp reads (5M pairs, insert N(300, 30)), 0.5 % errors.
    5  1,000 genomes of 1-6 Mbp, abundance log-normal(0, 2), 200M paired reads,
       1 % errors.

    ``scale`` < 1 shrinks the read count and the genome lengths together, so
    coverage and the count distribution keep their shape.
    """
    seed = BASE_SEED + 100 * i + seed_offset
    if i == 1:
        L = max(200, int(round(50_000 * scale)))
        g, off = genomes(seed, [L], [0.5])
        n = max(1, int(round(6_667 * scale)))
        r = simulate(seed, g, off, [1.0], n, paired=False, p_err=0.005)
    elif i == 2 or i == 5:
        if i == 2:
            ng, lo, hi, sig, npairs, perr = 100, 2_000_000, 5_000_000, 1.5, 5_000_000, 0.005
        else:
            ng, lo, hi, sig, npairs, perr = 1000, 1_000_000, 6_000_000, 2.0, 100_000_000, 0.01
        lengths, gcs, ab = metagenome(seed, ng, lo, hi, 0.3, 0.7, sig)
        lengths = np.maximum(1000, np.round(lengths * scale)).astype(np.int64)
        g, off = genomes(seed, lengths, gcs)
        n = max(1, int(round(npairs * scale)))
        r = simulate(seed, g, off, ab, n, paired=True, p_err=perr)
    else:
        raise ValueError("no read set for workload %d" % i)
    r.meta.update(config=i, scale=scale)
    return r


def serving_samples(n_samples: int = 64, reads_per_genome: int = 100_000,
                    scale: float = 1.0, seed_offset: int = 0):
    """Per-sample metagenomes for the serving workload: each sample has
    U{5..40} genomes drawn as in workload 2 and 0.1M x #genomes paired reads
    (times ``scale``).  Returns a list of (genome parameters, read count)."""
    seed = BASE_SEED + 400 + seed_offset
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_samples):
        ng = int(rng.integers(5, 41))
        lengths, gcs, ab = metagenome(seed * 1000 + s, ng, 2_000_000, 5_000_000,
                                      0.3, 0.7, 1.5)
        lengths = np.maximum(1000, np.round(lengths * scale)).astype(np.int64)
        out.append(dict(sample=s, seed=seed * 1000 + s, lengths=lengths,
                        gcs=gcs, abundance=ab,
                        n_reads=max(2, int(round(reads_per_genome * ng * scale)))))
    return out


def sample_reads(spec: dict) -> Reads:
    """Materialise the reads of one serving sample from ``serving_samples``."""
    g, off = genomes(spec["seed"], spec["lengths"], spec["gcs"])
    r = simulate(spec["seed"], g, off, spec["abundance"], spec["n_reads"] // 2,
                 paired=True, p_err=0.005)
    r.meta.update(sample=spec["sample"])
    return r
