"""Pins for the pruning oracle (Algorithm 2, iterative graph pruning): an
independent brute force on contigs of random read sets, closed forms (a
low-depth tip and a low-depth bubble branch beside a deep genome go at the
first sweep whose threshold reaches their depth; the genome's pieces stay),
invariants, and planted mistakes the brute force catches."""
import math

import numpy as np
import pytest

import brute
import oracle
import synth
from test_traverse_pins import _no_repeat, _random_genome, _tile


def _random_contigs(seed):
    """Contigs of a random read set: reads with errors, uneven coverage."""
    rng = np.random.default_rng(5000 + seed)
    k = int(rng.choice([5, 7, 11, 21]))
    g = _random_genome(rng, int(rng.integers(60, 500)))
    pairs = []
    for _ in range(int(rng.integers(20, 200))):
        a = int(min(len(g) - 10, abs(rng.normal(0.3, 0.3)) * len(g)))
        s = list(g[a:a + int(rng.integers(k, 70))])
        for i in range(len(s)):
            if rng.random() < 0.02:
                s[i] = "ACGT"[int(rng.integers(0, 4))]
        s = "".join(s)
        if rng.random() < 0.5:
            s = brute.revcomp(s)
        pairs.append((s, "I" * len(s)))
    t = oracle.count(synth.Reads.from_strings(pairs), k, min_count=int(rng.integers(1, 3)))
    c = oracle.traverse(t)
    alpha = float(rng.choice([0.05, 0.1, 0.3, 1.0]))
    beta = float(rng.choice([0.1, 0.2, 0.5, 1.0, 2.0]))
    return c, k, alpha, beta


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_random(seed):
    c, k, alpha, beta = _random_contigs(seed)
    got, sweeps = oracle.prune(c["seqs"], k, c["depth"], alpha, beta)
    want, want_sweeps = brute.prune(c["seqs"], k, c["depth"], alpha, beta)
    assert list(got) == want
    assert sweeps == want_sweeps


def test_random_cases_prune_something():
    """The random cases exercise removals, not only the empty outcome."""
    removed = 0
    for seed in range(40):
        c, k, alpha, beta = _random_contigs(seed)
        got, _ = oracle.prune(c["seqs"], k, c["depth"], alpha, beta)
        removed += int((got >= 0).sum())
    assert removed > 20


@pytest.mark.parametrize("seed", range(10))
def test_invariants(seed):
    c, k, alpha, beta = _random_contigs(seed)
    seqs, depth = c["seqs"], c["depth"]
    got, _ = oracle.prune(seqs, k, depth, alpha, beta)
    near = brute.prune_neighbours(seqs, k)
    for i, s in enumerate(seqs):
        if len(s) > 2 * k or not near[i]:
            assert got[i] == -1  # long, or nothing to compare with: stays
    zero, _ = oracle.prune(seqs, k, depth, alpha, 0.0)
    assert np.all(zero == -1)  # beta = 0: nothing of positive depth goes
    # one sweep at tau = 1, then tau = 1001 is beyond every depth: only
    # contigs of mean depth <= 1 can go, and only in that sweep
    mean = np.array([float(d) / n for d, n in zip(depth, c["n_kmers"])])
    assert mean.max() < 1001
    big, sweeps = oracle.prune(seqs, k, depth, 1000.0, beta)
    assert sweeps <= 1 and np.all(big <= 0) and np.all(mean[big == 0] <= 1.0)


def _sweep_reaching(d, alpha):
    """First sweep whose threshold (1 + alpha)^i reaches depth d."""
    return math.ceil(math.log(d) / math.log(1.0 + alpha))


def test_tip_goes_at_its_depth():
    rng = np.random.default_rng(21)
    k, alpha, beta = 21, 0.1, 0.2
    p = 450
    while True:
        g = _random_genome(rng, 900)
        y = _random_genome(rng, 5)
        v = g[p - 30:p] + y
        if y[0] != g[p] and _no_repeat(g, k - 1) and _no_repeat(g[:p] + y, k - 1):
            break
    t = oracle.count(synth.Reads.from_strings(
        [(s, "I" * len(s)) for s in _tile(g) for _ in range(2)] + [(v, "I" * len(v))] * 3), k)
    c = oracle.traverse(t)
    got, sweeps = oracle.prune(c["seqs"], k, c["depth"], alpha, beta)
    tv = g[p - k + 1:p] + y  # the tip: its k-mers are those holding a base of y
    tip = [i for i, s in enumerate(c["seqs"]) if s in (tv, brute.revcomp(tv))]
    assert len(tip) == 1
    assert int(c["depth"][tip[0]]) == 3 * 5
    assert got[tip[0]] == _sweep_reaching(3.0, alpha)
    kept = [s for i, s in enumerate(c["seqs"]) if got[i] < 0]
    # the genome splits at the fork into two pieces that cover it and stay
    assert sorted(kept) == sorted(min(x, brute.revcomp(x)) for x in (g[:p], g[p - k + 1:]))
    md = max(float(d) / n for d, n in zip(c["depth"], c["n_kmers"]))
    assert sweeps == _sweep_reaching(md, alpha)


def test_bubble_branch_goes_genome_side_stays():
    rng = np.random.default_rng(22)
    k, alpha, beta = 21, 0.1, 0.2
    p = 450
    while True:
        g = _random_genome(rng, 900)
        x = "ACGT"[int(rng.integers(0, 4))]
        gv = g[:p] + x + g[p + 1:]
        branch = gv[p - k + 1:p + k]
        novel = all(branch[i:i + k - 1] not in g and brute.revcomp(branch[i:i + k - 1]) not in g
                    for i in range(1, k))  # (k-1)-mers holding the variant base
        if x != g[p] and _no_repeat(g, k - 1) and novel and _no_repeat(branch, k - 1):
            break
    v = gv[p - 30:p + 31]
    t = oracle.count(synth.Reads.from_strings(
        [(s, "I" * len(s)) for s in _tile(g) for _ in range(2)] + [(v, "I" * len(v))] * 3), k)
    c = oracle.traverse(t)
    got, _ = oracle.prune(c["seqs"], k, c["depth"], alpha, beta)
    var = gv[p - k + 1:p + k]  # the 2k-1 bases of the variant branch
    vi = [i for i, s in enumerate(c["seqs"]) if s in (var, brute.revcomp(var))]
    assert len(vi) == 1 and int(c["depth"][vi[0]]) == 3 * k
    assert got[vi[0]] == _sweep_reaching(3.0, alpha)
    kept = sorted(s for i, s in enumerate(c["seqs"]) if got[i] < 0)
    # left piece, the genome's own (short, deep) branch, right piece
    want = (g[:p], g[p - k + 1:p + k], g[p + 1:])
    assert kept == sorted(min(s, brute.revcomp(s)) for s in want)


def test_hand_example():
    """A deep contig with two short neighbours of depth 2 and 9: with
    beta = 0.2 the pooled neighbourhood depth 300/11 gives a cut of 5.45, so
    the depth-2 tip goes at the first tau >= 2 (1.1^8) and the depth-9 one
    never; 35 sweeps bring tau past 27.3."""
    main = "AAACCCAGGATTTGC"  # 11 5-mers, depth 300 in all
    tips = ["CAGGTT", "TTGCAC"]  # each 2 5-mers, overlapping main by 4 bases
    got, sweeps = oracle.prune([main] + tips, 5, [300, 4, 18], 0.1, 0.2)
    assert list(got) == [-1, 8, -1]
    assert sweeps == 35


def test_oracle_rejects_bad_input():
    with pytest.raises(ValueError):
        oracle.prune(["ACGTACGTAC"], 5, [3])  # a 5-mer twice (reverse complements)
    with pytest.raises(ValueError):
        oracle.prune(["ACNTTGG"], 5, [3])
    with pytest.raises(ValueError):
        oracle.prune(["ACG"], 5, [3])  # shorter than k
    with pytest.raises(ValueError):
        oracle.prune(["AAACCCAGG"], 5, [3], alpha=0.0)


@pytest.mark.parametrize("mistake", [dict(synchronous=False), dict(pooled=False)])
def test_brute_force_sees_planted_mistakes(mistake):
    differs = 0
    for seed in range(40):
        c, k, alpha, beta = _random_contigs(seed)
        a = brute.prune(c["seqs"], k, c["depth"], alpha, beta)
        b = brute.prune(c["seqs"], k, c["depth"], alpha, beta, **mistake)
        differs += int(a != b)
    assert differs > 0
