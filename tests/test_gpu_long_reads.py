"""Reads far longer than a tile (assembled contigs, long reads): every
window of a read that spans tens of tiles, and reads longer than one block's
staging buffer in the minimizer reorder, against the oracle."""
import numpy as np
import pytest

import brute
import oracle
import synth
from brute import assert_same_table
from test_traverse_pins import _random_genome

pytestmark = pytest.mark.gpu


def _long_reads(seed):
    rng = np.random.default_rng(seed)
    g = _random_genome(rng, 120_000)
    pairs = []
    for _ in range(14):
        n = int(rng.integers(2_000, 60_000))
        a = int(rng.integers(0, len(g) - n))
        s = list(g[a:a + n])
        for i in rng.choice(n, size=n // 500, replace=False):  # sequencing errors
            s[i] = "ACGT"[(("ACGT".index(s[i])) + int(rng.integers(1, 4))) % 4]
        for i in rng.choice(n, size=3, replace=False):  # a few ambiguous bases
            s[i] = "N"
        s = "".join(s)
        q = "".join(chr(33 + int(x)) for x in rng.integers(2, 42, size=n))
        pairs.append((brute.revcomp(s) if rng.random() < 0.5 else s, q))
    pairs += [("ACGTTGCA" * 5, "I" * 40), ("", "")]  # short and empty among them
    return synth.Reads.from_strings(pairs)


@pytest.fixture(scope="module")
def lctx(kh):
    c = kh.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("k", [21, 77, 127])
@pytest.mark.parametrize("bloom", [False, True])
def test_single_k(lctx, k, bloom):
    reads = _long_reads(11)
    got = lctx.count(reads, k, use_bloom=bloom, min_count=2)
    assert_same_table(got.to_numpy(), oracle.count(reads, k, min_count=2))
    got.free()


def test_batched_and_aggregating(kh, lctx):
    reads = _long_reads(12)
    ks = [21, 33, 55, 99]
    want = {k: oracle.count(reads, k) for k in ks}
    for aggregate in (0, 1):
        lctx.set_tuning(aggregate=aggregate)
        tabs = lctx.count_multi_k(kh.DeviceReads.from_host(reads), ks, use_bloom=True)
        for k, t in zip(ks, tabs):
            assert_same_table(t.to_numpy(), want[k])
            t.free()
    lctx.set_tuning(aggregate=0)
