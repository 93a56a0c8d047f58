"""Merging earlier contigs' k-mers into a table on the GPU, against the
merge oracle on the same table (the GPU table is exported and merged by the
oracle, so the check isolates the merge)."""
import numpy as np
import pytest

import brute
import oracle
import synth
from brute import assert_same_table
from test_merge_pins import _random_case
from test_traverse_pins import _no_repeat, _random_genome

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mctx(kh):
    c = kh.Context(0)
    yield c
    c.close()


def _check(mctx, table, contigs, seqs=None):
    t = table.to_numpy()
    got = mctx.merge_contigs(table, contigs).to_numpy()
    want = oracle.merge(t, seqs if seqs is not None else contigs)
    print("k=%d rows %d -> %d" % (t["k"], t["n_rows"], want["n_rows"]), flush=True)
    assert_same_table(got, want, totals=False)
    assert got["n_windows"] == t["n_windows"]
    return got


@pytest.mark.parametrize("seed", range(20))
def test_random_tables_and_contigs(mctx, seed):
    _, contigs, reads, mc = _random_case(seed)
    k = _random_case(seed)[0]["k"]
    _check(mctx, mctx.count(reads, k, min_count=mc), contigs)


@pytest.mark.parametrize("k0,k1", [(21, 33), (33, 55), (55, 99)])
def test_contigs_of_the_previous_k(mctx, k0, k1):
    """Algorithm 1's loop: contigs at k0, merged into the k1 table on the
    device (the Contigs object is used in place)."""
    reads = synth.config(1, scale=0.5)
    c = mctx.traverse(mctx.count(reads, k0))
    seqs = c.to_python()["seqs"]
    _check(mctx, mctx.count(reads, k1, min_count=3), c, seqs)


def test_metagenome_sample(mctx):
    reads = synth.config(2, scale=0.01)
    c = mctx.traverse(mctx.count(reads, 21, use_bloom=True))
    seqs = c.to_python()["seqs"]
    got = _check(mctx, mctx.count(reads, 33, use_bloom=True), c, seqs)
    assert np.any(got["counts"] == 0)  # contig k-mers the reads alone lost


def test_round_trip_through_traversal(mctx):
    rng = np.random.default_rng(12)
    k = 21
    while True:
        g = _random_genome(rng, 500)
        if _no_repeat(g, k - 1):
            break
    empty = synth.Reads(np.zeros(0, np.uint8), np.zeros(0, np.uint8), np.zeros(1, np.int64))
    m = mctx.merge_contigs(mctx.count(empty, k), [g])
    c = mctx.traverse(m).to_python()
    assert c["seqs"] == [min(g, brute.revcomp(g))]
    assert int(c["depth"][0]) == 0


def test_errors(kh, mctx):
    t = mctx.count(synth.config(1, scale=0.1), 21)
    got = mctx.merge_contigs(t, []).to_numpy()  # nothing to merge
    assert_same_table(got, t.to_numpy(), totals=False)


def test_pipeline_matches_the_oracle_chain(kh, mctx):
    """Algorithm 1's in-scope steps over k = 21, 33, 55 (table, merge of the
    previous pruned contigs, traversal, pruning) equal the same chain of
    oracle calls."""
    from paper_1809_07014_amd import pipeline
    reads = synth.config(1, scale=0.5)
    ks = [21, 33, 55]
    last, reports = pipeline.iterate(mctx, reads, ks)
    got = last.to_python()
    last.free()
    prev = None
    for k in ks:
        t = oracle.count(reads, k)
        if prev is not None:
            t = oracle.merge(t, prev)
        walked = oracle.traverse(t)
        removed, sweeps = oracle.prune(walked["seqs"], k, walked["depth"])
        keep = removed < 0
        want = dict(seqs=[x for x, y in zip(walked["seqs"], keep) if y],
                    depth=walked["depth"][keep])
        rep = reports[len([x for x in ks if x < k])]
        assert (rep["n_contigs"], rep["pruned"], rep["sweeps"]) == (
            walked["n_contigs"], int((~keep).sum()), sweeps)
        prev = want["seqs"]
    assert got["seqs"] == want["seqs"]
    np.testing.assert_array_equal(got["depth"], want["depth"])
    assert [r["k"] for r in reports] == ks
