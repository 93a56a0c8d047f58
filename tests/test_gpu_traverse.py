"""Contigs on the GPU (de Bruijn graph traversal) against the contig oracle,
on the same table: the GPU table is exported and traversed by the oracle, so
the check isolates the traversal (counting parity is tested elsewhere)."""
import numpy as np
import pytest

import brute
import oracle
import synth
from test_traverse_pins import _no_repeat, _random_genome, _reads, _tile

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tctx(kh):
    c = kh.Context(0)
    yield c
    c.close()


def _gpu_contigs(tctx, table):
    c = tctx.traverse(table)
    got = c.to_python()
    info = c.info()
    c.free()
    return got, info


def _check(tctx, table):
    t = table.to_numpy()
    got, info = _gpu_contigs(tctx, table)
    want = oracle.traverse(t)
    print("k=%d rows=%d contigs=%d rounds=%d cycle_kmers=%d" % (
        t["k"], t["n_rows"], want["n_contigs"], info["rounds"], info["cycle_kmers"]), flush=True)
    assert got["n_contigs"] == want["n_contigs"]
    assert got["seqs"] == want["seqs"]
    np.testing.assert_array_equal(got["n_kmers"], want["n_kmers"])
    np.testing.assert_array_equal(got["depth"], want["depth"])
    np.testing.assert_array_equal(got["cycle"], want["cycle"])
    assert int(got["n_kmers"].sum()) == t["n_rows"]
    return got


@pytest.mark.parametrize("k", [21, 33, 55, 77, 99, 127])
def test_small_workload(tctx, k):
    _check(tctx, tctx.count(synth.config(1), k))


@pytest.mark.parametrize("k", [21, 55])
def test_metagenome_sample(tctx, k):
    reads = synth.config(2, scale=0.01)
    _check(tctx, tctx.count(reads, k, use_bloom=True))


@pytest.mark.parametrize("seed", range(12))
def test_random_tiny_tables(tctx, seed):
    rng = np.random.default_rng(2000 + seed)
    k = int(rng.choice([3, 5, 7, 9, 11]))
    g = _random_genome(rng, int(rng.integers(30, 300)))
    pairs = []
    for _ in range(int(rng.integers(5, 80))):
        a = int(rng.integers(0, max(1, len(g) - 10)))
        s = list(g[a:a + int(rng.integers(k, 60))])
        for i in range(len(s)):
            if rng.random() < 0.03:
                s[i] = "ACGT"[int(rng.integers(0, 4))]
        s = "".join(s)
        if rng.random() < 0.5:
            s = brute.revcomp(s)
        pairs.append((s, "".join(chr(33 + int(x)) for x in rng.integers(2, 42, size=len(s)))))
    reads = synth.Reads.from_strings(pairs)
    got = _check(tctx, tctx.count(reads, k, min_count=int(rng.integers(1, 3)),
                                  t_min_ext=int(rng.integers(1, 3))))
    assert got["n_contigs"] >= 1


def test_circular_genome(tctx):
    rng = np.random.default_rng(7)
    k = 21
    while True:
        g = _random_genome(rng, 600)
        if _no_repeat(g, k - 1, circular=True):
            break
    got = _check(tctx, tctx.count(_reads(_tile(g, circular=True)), k))
    assert got["n_contigs"] == 1 and bool(got["cycle"][0])
    assert len(got["seqs"][0]) == len(g) + k - 1


def test_planted_repeat(tctx):
    rng = np.random.default_rng(9)
    k = 21
    while True:
        X, Y, Z = (_random_genome(rng, 200) for _ in range(3))
        R = _random_genome(rng, 60)
        if X[-1] != Y[-1] and Y[0] != Z[0] and _no_repeat(X + R + Y + Z, k - 1) \
                and _no_repeat(R + Z, k - 1):
            break
    got = _check(tctx, tctx.count(_reads(_tile(X + R + Y + R + Z)), k))
    j = k - 1
    want = sorted(min(s, brute.revcomp(s)) for s in
                  (X + R[:j], R, R[-j:] + Y + R[:j], R[-j:] + Z))
    assert sorted(got["seqs"]) == want


def test_edge_tables(kh, tctx):
    empty = synth.Reads(np.zeros(0, np.uint8), np.zeros(0, np.uint8), np.zeros(1, np.int64))
    got, info = _gpu_contigs(tctx, tctx.count(empty, 21))
    assert got["n_contigs"] == 0 and info["total_bases"] == 0
    one = synth.Reads.from_strings([("ACGTACGTTGCA" * 2, "I" * 24)] * 2)
    _check(tctx, tctx.count(one, 23))


def test_table_of_destroyed_context(kh):
    c1 = kh.Context(0)
    t = c1.count(synth.config(1, scale=0.1), 21)
    c1.close()
    c2 = kh.Context(0)
    with pytest.raises(kh.KHError) as e:
        c2.traverse(t)
    assert e.value.code == kh.KH_EINVAL
    t.free()
    c2.close()
