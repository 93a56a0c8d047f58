"""Iterative graph pruning on the GPU (Algorithm 2) against the pruning
oracle: the GPU table is traversed on the GPU, pruned on the GPU, and the
same contigs are pruned by the oracle; the sweep that removed each contig,
the number of sweeps and the kept contigs must agree exactly."""
import numpy as np
import pytest

import brute
import oracle
import synth
from test_traverse_pins import _no_repeat, _random_genome, _tile

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pctx(kh):
    c = kh.Context(0)
    yield c
    c.close()


def _check(pctx, table, alpha=0.1, beta=0.2):
    c = pctx.traverse(table)
    cont = c.to_python()
    kept, rep, removed = pctx.prune(table, c, alpha=alpha, beta=beta, removed_at=True)
    got = kept.to_python()
    kept.free()
    c.free()
    want, sweeps = oracle.prune(cont["seqs"], cont["k"], cont["depth"], alpha, beta)
    print("k=%d contigs=%d removed=%d sweeps=%d" % (cont["k"], cont["n_contigs"],
                                                   int((want >= 0).sum()), sweeps), flush=True)
    np.testing.assert_array_equal(removed, want)
    assert rep["sweeps"] == sweeps
    assert rep["removed"] == int((want >= 0).sum())
    keep = want < 0
    assert got["seqs"] == [s for s, x in zip(cont["seqs"], keep) if x]
    np.testing.assert_array_equal(got["n_kmers"], cont["n_kmers"][keep])
    np.testing.assert_array_equal(got["depth"], cont["depth"][keep])
    np.testing.assert_array_equal(got["cycle"], cont["cycle"][keep])
    if keep.any():
        md = max(float(d) / n for d, n in zip(got["depth"], got["n_kmers"]))
        assert rep["max_depth"] == md and not rep["tau"] < md
    return want


def _reads_with_errors(rng, k, n_reads, err=0.02):
    g = _random_genome(rng, int(rng.integers(200, 2000)))
    pairs = []
    for _ in range(n_reads):
        a = int(min(len(g) - 10, abs(rng.normal(0.3, 0.3)) * len(g)))
        s = list(g[a:a + int(rng.integers(k, 150))])
        for i in range(len(s)):
            if rng.random() < err:
                s[i] = "ACGT"[int(rng.integers(0, 4))]
        s = "".join(s)
        if rng.random() < 0.5:
            s = brute.revcomp(s)
        pairs.append((s, "I" * len(s)))
    return synth.Reads.from_strings(pairs)


@pytest.mark.parametrize("seed", range(16))
def test_random_read_sets(pctx, seed):
    rng = np.random.default_rng(6000 + seed)
    k = int(rng.choice([5, 7, 11, 21, 33, 55, 77, 99]))
    reads = _reads_with_errors(rng, k, int(rng.integers(50, 800)))
    alpha = float(rng.choice([0.05, 0.1, 0.3, 1.0]))
    beta = float(rng.choice([0.1, 0.2, 0.5, 1.0, 2.0]))
    _check(pctx, pctx.count(reads, k, min_count=int(rng.integers(1, 3))), alpha, beta)


def test_random_read_sets_remove_something(pctx):
    removed = 0
    for seed in range(4):
        rng = np.random.default_rng(6100 + seed)
        reads = _reads_with_errors(rng, 21, 1500, err=0.01)
        removed += int((_check(pctx, pctx.count(reads, 21)) >= 0).sum())
    assert removed > 0


@pytest.mark.parametrize("k", [21, 33])
def test_metagenome_sample(pctx, k):
    reads = synth.config(2, scale=0.01)
    _check(pctx, pctx.count(reads, k, use_bloom=True))


@pytest.mark.parametrize("k", [21, 55, 99])
def test_small_workload(pctx, k):
    _check(pctx, pctx.count(synth.config(1), k))


def test_tip_on_the_gpu(pctx):
    rng = np.random.default_rng(21)
    k, p = 21, 450
    while True:
        g = _random_genome(rng, 900)
        y = _random_genome(rng, 5)
        v = g[p - 30:p] + y
        if y[0] != g[p] and _no_repeat(g, k - 1) and _no_repeat(g[:p] + y, k - 1):
            break
    reads = synth.Reads.from_strings(
        [(s, "I" * len(s)) for s in _tile(g) for _ in range(2)] + [(v, "I" * len(v))] * 3)
    removed = _check(pctx, pctx.count(reads, k))
    assert int((removed >= 0).sum()) == 1


def test_edge_cases(kh, pctx):
    # a table with no rows
    t = pctx.count(synth.Reads.from_strings([("ACGTA", "IIIII")]), 21)
    c = pctx.traverse(t)
    kept, rep, removed = pctx.prune(t, c, removed_at=True)
    assert kept.info()["n_contigs"] == 0 and rep["sweeps"] == 0 and len(removed) == 0
    kept.free()
    # one contig: nothing to compare with, never removed
    rng = np.random.default_rng(5)
    g = _random_genome(rng, 40)
    t1 = pctx.count(synth.Reads.from_strings([(g, "I" * 40)] * 3), 21)
    c1 = pctx.traverse(t1)
    kept, rep, removed = pctx.prune(t1, c1, removed_at=True)
    assert list(removed) == [-1] and rep["sweeps"] == 12  # 1.1^11 < 3 <= 1.1^12
    kept.free()
    # contigs walked from another table, parameters out of range
    with pytest.raises(kh.KHError):
        pctx.prune(t, c1)
    with pytest.raises(kh.KHError):
        pctx.prune(t1, c1, alpha=0.0)
    with pytest.raises(kh.KHError):
        pctx.prune(t1, c1, beta=-1.0)
    # pruned contigs carry no row map: they cannot be pruned again
    kept, _ = pctx.prune(t1, c1)
    with pytest.raises(kh.KHError):
        pctx.prune(t1, kept)
    kept.free()
    for x in (c, c1):
        x.free()
    for x in (t, t1):
        x.free()
