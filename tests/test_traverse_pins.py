"""Pins for the contig oracle (de Bruijn graph traversal, paper Section
II-C): an independent brute force on random tiny tables, and three read sets
whose contigs are known in closed form (a circular genome, an error-free
linear genome, a genome with a planted repeat)."""
import numpy as np
import pytest

import brute
import oracle
import synth


def _as_list(c):
    return [(c["seqs"][i], int(c["n_kmers"][i]), int(c["depth"][i]), bool(c["cycle"][i]))
            for i in range(c["n_contigs"])]


def _reads(strings, copies=2):
    pairs = [(s, "I" * len(s)) for s in strings for _ in range(copies)]
    return synth.Reads.from_strings(pairs)


def _tile(genome, L=50, circular=False):
    g = genome + genome[:L - 1] if circular else genome
    n = len(genome) if circular else len(genome) - L + 1
    return [g[p:p + L] for p in range(n)]


def _random_genome(rng, n):
    return "".join(rng.choice(list("ACGT"), size=n))


def _no_repeat(s, m, circular=False):
    """No m-mer occurs twice (on either strand) in s (read around the circle
    if circular)."""
    ext = s + s[:m - 1] if circular else s
    n = len(s) if circular else len(s) - m + 1
    seen = set()
    for i in range(n):
        w = ext[i:i + m]
        c = min(w, brute.revcomp(w))
        if c in seen:
            return False
        seen.add(c)
    return True


@pytest.mark.parametrize("seed", range(30))
def test_brute_force_random_tables(seed):
    rng = np.random.default_rng(1000 + seed)
    k = int(rng.choice([3, 5, 7, 11, 21]))
    g = _random_genome(rng, int(rng.integers(30, 400)))
    pairs = []
    for _ in range(int(rng.integers(5, 60))):
        a = int(rng.integers(0, max(1, len(g) - 10)))
        s = list(g[a:a + int(rng.integers(k, 60))])
        for i in range(len(s)):
            if rng.random() < 0.03:
                s[i] = "ACGT"[int(rng.integers(0, 4))]
        s = "".join(s)
        if rng.random() < 0.5:
            s = brute.revcomp(s)
        q = "".join(chr(33 + int(x)) for x in rng.integers(2, 42, size=len(s)))
        pairs.append((s, q))
    reads = synth.Reads.from_strings(pairs)
    kw = dict(min_count=int(rng.integers(1, 3)), t_min_ext=int(rng.integers(1, 3)),
              qual_cutoff=int(rng.integers(0, 30)))
    t = oracle.count(reads, k, **kw)
    got = _as_list(oracle.traverse(t))
    want = brute.contigs(t)
    assert got == want
    assert sum(x[1] for x in got) == t["n_rows"]


def test_circular_genome_is_one_cycle():
    rng = np.random.default_rng(7)
    k = 21
    while True:
        g = _random_genome(rng, 600)
        if _no_repeat(g, k - 1, circular=True):
            break
    t = oracle.count(_reads(_tile(g, circular=True)), k)
    assert t["n_rows"] == len(g)
    c = _as_list(oracle.traverse(t))
    assert len(c) == 1
    seq, nk, depth, cyc = c[0]
    assert cyc and nk == len(g) and len(seq) == len(g) + k - 1
    # opened at the smallest canonical k-mer, read in its canonical orientation
    m = brute.key_text(t["keys"][0], k)
    src = g if (g + g).find(m) >= 0 else brute.revcomp(g)
    p = (src + src).find(m)
    assert seq == (src * 3)[p:p + len(g) + k - 1]
    assert depth == int(t["counts"].sum())


def test_linear_genome_is_one_contig():
    rng = np.random.default_rng(8)
    k = 21
    while True:
        g = _random_genome(rng, 800)
        if _no_repeat(g, k - 1):
            break
    t = oracle.count(_reads(_tile(g)), k)
    c = _as_list(oracle.traverse(t))
    assert c == [(min(g, brute.revcomp(g)), len(g) - k + 1, int(t["counts"].sum()), False)]


def test_planted_repeat_gives_four_contigs():
    rng = np.random.default_rng(9)
    k = 21
    while True:
        X, Y, Z = (_random_genome(rng, 200) for _ in range(3))
        R = _random_genome(rng, 60)
        g = X + R + Y + R + Z
        ok = X[-1] != Y[-1] and Y[0] != Z[0]
        # no (k-1)-mer repeats except inside the two copies of R
        if ok and _no_repeat(X + R + Y + Z, k - 1) and _no_repeat(R + Z, k - 1):
            break
    t = oracle.count(_reads(_tile(g)), k)
    got = sorted(s for s, _, _, _ in _as_list(oracle.traverse(t)))
    j = k - 1
    want = sorted(min(s, brute.revcomp(s)) for s in
                  (X + R[:j], R, R[-j:] + Y + R[:j], R[-j:] + Z))
    assert got == want


def test_brute_force_is_sensitive_to_mutuality():
    """Dropping the mutual-edge condition (a plausible mistake) changes the
    planted-repeat contigs: the brute force would catch it."""
    rng = np.random.default_rng(9)
    X, Y, Z = (_random_genome(rng, 200) for _ in range(3))
    R = _random_genome(rng, 60)
    t = oracle.count(_reads(_tile(X + R + Y + R + Z)), 21)
    with pytest.raises(AssertionError):
        assert brute.contigs(t, mutual=False) == brute.contigs(t)
