"""The export sort on tables large enough for its segmented path (rows put
in the order of their top key bits, then runs of buckets sorted in LDS):
about 1.7M rows per k, keys of one to three words (k = 21, 25 and 31 sort
whole keys of 42, 50 and 62 bits; k = 33 and 77 sort 40-bit prefixes and
order equal prefixes by the full key), against the oracle row for row.  A
planted bucket holds more rows than one LDS segment: 30,000 distinct
k-mers that share their first five bases (each read twice), which the
plain radix passes sort on their own."""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle
import synth
from brute import assert_same_table

pytestmark = pytest.mark.gpu

KS = (21, 25, 31, 33, 77)


def _reads():
    base = synth.config(2, scale=0.01)  # 100,000 reads
    rng = np.random.default_rng(77)
    pairs = []
    for k in (21,):
        for _ in range(30_000):
            s = "AAAAA" + "".join(rng.choice(list("CGT"), size=1)) + \
                "".join(rng.choice(list("ACGT"), size=k - 6))
            pairs += [(s, "I" * k)] * 2
    extra = synth.Reads.from_strings(pairs)
    seq = np.concatenate([base.seq, extra.seq])
    qual = np.concatenate([base.qual, extra.qual])
    off = np.concatenate([base.offsets, extra.offsets[1:] + base.offsets[-1]])
    return synth.Reads(seq, qual, off)


@pytest.fixture(scope="module")
def data():
    reads = _reads()
    with cf.ThreadPoolExecutor(max_workers=min(len(KS), os.cpu_count() or 1)) as ex:
        want = dict(zip(KS, ex.map(lambda k: oracle.count(reads, k), KS)))
    return reads, want


@pytest.mark.parametrize("bloom", [False, True])
def test_segmented_sort_matches_oracle(kh, data, bloom):
    reads, want = data
    ctx = kh.Context(0)
    try:
        dev = kh.DeviceReads.from_host(reads)
        for k in KS:  # single-k path
            got = ctx.count(dev, k, use_bloom=bloom).to_numpy()
            print("k=%d rows=%d" % (k, got["n_rows"]), flush=True)
            assert got["n_rows"] > 1_000_000
            assert_same_table(got, want[k])
        tabs = ctx.count_multi_k(dev, KS, use_bloom=bloom)  # batched path
        for k, t in zip(KS, tabs):
            assert_same_table(t.to_numpy(), want[k])
    finally:
        ctx.close()
