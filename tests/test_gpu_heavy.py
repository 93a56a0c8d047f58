"""Heavy-hitter reporting on the GPU: the rows at or above a count threshold
equal the oracle table's rows at or above it (the plain definition), also
for k-mers beyond the 4096 occurrences that take the exact recount path."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hctx(kh):
    c = kh.Context(0)
    yield c
    c.close()


def _want(t, h):
    sel = t["counts"] >= h
    return t["keys"][sel], t["counts"][sel]


def test_planted_heavy_kmers(hctx):
    rng = np.random.default_rng(3)
    hot = "".join(rng.choice(list("ACGT"), 150))
    pairs = [(hot, "I" * 150)] * 5000
    for _ in range(2000):
        s = "".join(rng.choice(list("ACGT"), 150))
        pairs.append((s, "I" * 150))
    reads = synth.Reads.from_strings(pairs)
    for k in (21, 55):
        t = hctx.count(reads, k)
        want = oracle.count(reads, k)
        for h in (2, 4096, 5000, 5001):
            keys, counts = t.heavy_hitters(h)
            wk, wc = _want(want, h)
            np.testing.assert_array_equal(keys, wk)
            np.testing.assert_array_equal(counts, wc)
        assert len(t.heavy_hitters(4096)[1]) == len(want["counts"][want["counts"] >= 5000]) > 0
        t.free()


@pytest.mark.parametrize("h", [2, 30, 300])
def test_metagenome_sample(hctx, h):
    reads = synth.config(2, scale=0.01)
    t = hctx.count(reads, 33, use_bloom=True)
    keys, counts = t.heavy_hitters(h)
    wk, wc = _want(oracle.count(reads, 33), h)
    np.testing.assert_array_equal(keys, wk)
    np.testing.assert_array_equal(counts, wc)
    t.free()


def test_partial_copy_and_errors(kh, hctx):
    reads = synth.config(1, scale=0.2)
    t = hctx.count(reads, 21)
    want = oracle.count(reads, 21)
    wk, wc = _want(want, 3)
    keys = np.zeros((5, 1), np.uint64)
    counts = np.zeros(5, np.uint32)
    n = ctypes.c_int64()
    lib = kh.load()
    assert lib.kh_heavy_hitters(t.handle, 3, None, keys.ctypes.data, counts.ctypes.data, 5,
                                ctypes.byref(n)) == 0
    assert n.value == len(wc) > 5
    np.testing.assert_array_equal(keys, wk[:5])
    np.testing.assert_array_equal(counts, wc[:5])
    assert lib.kh_heavy_hitters(t.handle, 0, None, None, None, 0, ctypes.byref(n)) != 0
    assert lib.kh_heavy_hitters(t.handle, 3, None, None, None, 4, ctypes.byref(n)) != 0
    t.free()
    empty = hctx.count(synth.Reads.from_strings([("ACG", "III")]), 21)
    k2, c2 = empty.heavy_hitters(1)
    assert k2.shape == (0, 1) and len(c2) == 0
    empty.free()
