"""Pins for the merge oracle (Algorithm 1's Merge: earlier contigs' k-mers
join the k-mer table as error-free k-mers with unique extensions): an
independent brute force on random tables and contigs, and closed forms."""
import numpy as np
import pytest

import brute
import oracle
import synth
from brute import assert_same_table
from test_traverse_pins import _no_repeat, _random_genome


def _random_case(seed):
    rng = np.random.default_rng(3000 + seed)
    k = int(rng.choice([3, 5, 7, 11, 21, 33]))
    g = _random_genome(rng, int(rng.integers(40, 400)))
    pairs = []
    for _ in range(int(rng.integers(2, 40))):
        a = int(rng.integers(0, max(1, len(g) - 10)))
        s = g[a:a + int(rng.integers(k, 80))]
        if rng.random() < 0.5:
            s = brute.revcomp(s)
        pairs.append((s, "".join(chr(33 + int(x)) for x in rng.integers(2, 42, size=len(s)))))
    reads = synth.Reads.from_strings(pairs)
    mc = int(rng.integers(1, 4))
    t = oracle.count(reads, k, min_count=mc)
    contigs = []
    for _ in range(int(rng.integers(0, 8))):
        a = int(rng.integers(0, max(1, len(g) - 5)))
        c = list(g[a:a + int(rng.integers(1, 120))])
        for i in range(len(c)):
            u = rng.random()
            if u < 0.02:
                c[i] = "N"
            elif u < 0.05:
                c[i] = "ACGT"[int(rng.integers(0, 4))]
            elif u < 0.08:
                c[i] = c[i].lower()
        c = "".join(c)
        contigs.append(brute.revcomp(c.upper()) if rng.random() < 0.3 else c)
    return t, contigs, reads, mc


@pytest.mark.parametrize("seed", range(30))
def test_brute_force_random(seed):
    t, contigs, _, _ = _random_case(seed)
    got = oracle.merge(t, contigs)
    assert_same_table(got, brute.merge(t, contigs), totals=False)


def test_brute_force_sees_planted_mistake():
    """A merge that lets contig k-mers overwrite existing rows differs."""
    differs = 0
    for seed in range(30):
        t, contigs, _, _ = _random_case(seed)
        a, b = brute.merge(t, contigs), brute.merge(t, contigs, override=True)
        differs += int(not (np.array_equal(a["codes"], b["codes"])
                            and np.array_equal(a["counts"], b["counts"])))
    assert differs > 0


def test_one_contig_into_empty_table_walks_back():
    rng = np.random.default_rng(12)
    k = 21
    while True:
        g = _random_genome(rng, 500)
        if _no_repeat(g, k - 1):
            break
    empty = oracle.count(synth.Reads.from_strings([]), k)
    m = oracle.merge(empty, [g])
    assert m["n_rows"] == len(g) - k + 1
    assert int(m["counts"].sum()) == 0
    c = oracle.traverse(m)
    assert c["seqs"] == [min(g, brute.revcomp(g))]
    assert int(c["n_kmers"][0]) == len(g) - k + 1 and int(c["depth"][0]) == 0


def test_contigs_of_the_table_change_nothing():
    t = oracle.count(synth.config(1, scale=0.3), 21)
    c = oracle.traverse(t)
    m = oracle.merge(t, c["seqs"])
    assert_same_table(m, t, totals=False)
