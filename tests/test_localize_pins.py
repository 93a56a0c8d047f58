"""Pins for the read-localisation oracle (reads grouped by the contig their
first contig k-mer lies in): an independent brute force on random reads and
contigs, a closed form (reads tiled from several genomes and shuffled come
back grouped genome by genome), and the invariance that makes localisation a
pure performance variant (tables of the permuted reads equal the input's)."""
import numpy as np
import pytest

import brute
import oracle
import synth
from brute import assert_same_table
from test_traverse_pins import _no_repeat, _random_genome, _tile


def _reads_from(pairs):
    return synth.Reads.from_strings(pairs)


@pytest.mark.parametrize("seed", range(30))
def test_brute_force_random(seed):
    rng = np.random.default_rng(7000 + seed)
    k = int(rng.choice([3, 5, 7, 11, 21, 33]))
    g = _random_genome(rng, int(rng.integers(50, 600)))
    pairs = []
    for _ in range(int(rng.integers(0, 80))):
        a = int(rng.integers(0, max(1, len(g) - 10)))
        s = list(g[a:a + int(rng.integers(1, 90))])
        for i in range(len(s)):
            u = rng.random()
            if u < 0.02:
                s[i] = "N"
            elif u < 0.05:
                s[i] = "ACGT"[int(rng.integers(0, 4))]
            elif u < 0.08:
                s[i] = s[i].lower()
        s = "".join(s)
        if rng.random() < 0.4:
            s = brute.revcomp(s.upper())
        pairs.append((s, "I" * len(s)))
    contigs = []
    for _ in range(int(rng.integers(0, 10))):
        a = int(rng.integers(0, max(1, len(g) - 5)))
        c = g[a:a + int(rng.integers(1, 150))]
        contigs.append(brute.revcomp(c) if rng.random() < 0.3 else c)
    got = oracle.localize(_reads_from(pairs), contigs, k)
    want = brute.localize([s for s, _ in pairs], contigs, k)
    assert list(got) == want


def test_genomes_come_back_grouped():
    rng = np.random.default_rng(31)
    k = 21
    genomes = []
    while len(genomes) < 3:
        g = _random_genome(rng, 700)
        if _no_repeat("".join(genomes + [g]), k - 1):
            genomes.append(g)
    reads = [(s, gi) for gi, g in enumerate(genomes) for s in _tile(g, L=60)[::3]]
    reads += [(_random_genome(rng, 40), 3) for _ in range(25)]  # foreign sequence
    perm = rng.permutation(len(reads))
    reads = [reads[i] for i in perm]
    strand = rng.random(len(reads)) < 0.5
    pairs = [((brute.revcomp(s) if f else s), "I" * len(s)) for (s, _), f in zip(reads, strand)]
    t = oracle.count(_reads_from([(g, "I" * len(g)) for g in genomes] * 2), k)
    contigs = oracle.traverse(t)["seqs"]
    assert len(contigs) == 3
    which = [next(i for i, g in enumerate(genomes) if c in (g, brute.revcomp(g)))
             for c in contigs]
    order = oracle.localize(_reads_from(pairs), contigs, k)
    want = [i for gi in which + [3] for i in range(len(reads)) if reads[i][1] == gi]
    assert list(order) == want


@pytest.mark.parametrize("k", [21, 33])
def test_permuted_reads_give_the_same_table(k):
    reads = synth.config(1, scale=0.2)
    t = oracle.count(reads, 21)
    contigs = oracle.traverse(t)["seqs"]
    order = oracle.localize(reads, contigs, 21)
    assert sorted(order) == list(range(reads.n_reads))
    strings = reads.strings()
    moved = _reads_from([strings[i] for i in order])
    assert_same_table(oracle.count(moved, k), oracle.count(reads, k))


def test_edge_cases():
    reads = _reads_from([("ACGTTGCA", "IIIIIIII"), ("", ""), ("NNNN", "IIII")])
    assert list(oracle.localize(reads, [], 5)) == [0, 1, 2]
    assert list(oracle.localize(_reads_from([]), ["ACGTTGCAA"], 5)) == []
    # a read shorter than k has no anchor
    assert list(oracle.localize(_reads_from([("ACG", "III"), ("TTGCA", "IIIII")]),
                                ["ACGTTGCAA"], 5)) == [1, 0]
