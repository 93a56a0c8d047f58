"""The aggregating counting pass (tuning aggregate = 1: reads put in
minimizer order, each tile's repeated k-mers merged in LDS before one table
update per distinct k-mer) against the oracle: tables must be bit-identical,
including k-mers past the spill point of the packed counter and heavy
hitters, for one k at a time and for the batched call."""
import numpy as np
import pytest

import brute
import oracle
import synth
from brute import assert_same_table
from test_traverse_pins import _random_genome

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def actx(kh):
    c = kh.Context(0)
    c.set_tuning(aggregate=1)
    yield c
    c.close()


@pytest.mark.parametrize("k", [21, 33, 55, 77, 99])
def test_small_workload(actx, k):
    reads = synth.config(1)
    assert_same_table(actx.count(reads, k, use_bloom=True).to_numpy(), oracle.count(reads, k))


def test_metagenome_sample_batched(kh, actx):
    reads = synth.config(2, scale=0.02)
    ks = [21, 33, 55, 77, 99]
    tabs = actx.count_multi_k(kh.DeviceReads.from_host(reads), ks, use_bloom=True)
    for k, t in zip(ks, tabs):
        assert_same_table(t.to_numpy(), oracle.count(reads, k))
        t.free()


@pytest.mark.parametrize("tpb", [1, 3])
def test_deep_repeats_spill_and_heavy(actx, tpb):
    """A read repeated 5000 times (every k-mer heavy, every tile full of the
    same k-mers), a read repeated 70 times (past the spill point of the
    packed counter inside one tile), random reads around them."""
    actx.set_tuning(tiles_per_block=tpb)
    rng = np.random.default_rng(4)
    hot = _random_genome(rng, 150)
    warm = _random_genome(rng, 150)
    pairs = [(hot, "I" * 150)] * 5000 + [(warm, "I" * 75 + "#" * 75)] * 70
    for _ in range(3000):
        s = _random_genome(rng, int(rng.integers(30, 150)))
        pairs.append((brute.revcomp(s) if rng.random() < 0.5 else s, "I" * len(s)))
    order = rng.permutation(len(pairs))
    reads = synth.Reads.from_strings([pairs[i] for i in order])
    for k in (21, 33):
        assert_same_table(actx.count(reads, k, use_bloom=True).to_numpy(), oracle.count(reads, k))
    actx.set_tuning(tiles_per_block=4)


@pytest.mark.parametrize("seed", range(6))
def test_random_reads(actx, seed):
    rng = np.random.default_rng(8000 + seed)
    k = int(rng.choice([5, 11, 21, 31, 33, 63, 65, 127]))
    g = _random_genome(rng, int(rng.integers(200, 3000)))
    pairs = []
    for _ in range(int(rng.integers(50, 3000))):
        a = int(rng.integers(0, max(1, len(g) - 10)))
        s = list(g[a:a + int(rng.integers(1, 200))])
        for i in range(len(s)):
            u = rng.random()
            if u < 0.01:
                s[i] = "N"
            elif u < 0.03:
                s[i] = "ACGT"[int(rng.integers(0, 4))]
        s = "".join(s)
        q = "".join(chr(33 + int(x)) for x in rng.integers(2, 42, size=len(s)))
        pairs.append((brute.revcomp(s) if rng.random() < 0.5 else s, q))
    reads = synth.Reads.from_strings(pairs)
    mc = int(rng.integers(1, 3))
    got = actx.count(reads, k, use_bloom=mc >= 2, min_count=mc)
    assert_same_table(got.to_numpy(), oracle.count(reads, k, min_count=mc))


def test_rebuild_and_heavy_batched(actx, monkeypatch):
    """A table forced far too small (probe limit, rebuild) and homopolymer
    heavy hitters in the batched call with the aggregating pass."""
    pairs = [("A" * 100, "I" * 100)] * 900 + synth.config(1, scale=0.05).strings()
    reads = synth.Reads.from_strings(pairs)
    ks = [21, 33, 55, 77]
    want = {k: oracle.count(reads, k) for k in ks}
    monkeypatch.setenv("KMERHIP_FORCE_CAPACITY", "500")
    tabs = actx.count_multi_k(reads, ks, use_bloom=True)
    for i, (k, t) in enumerate(zip(ks, tabs)):
        assert_same_table(t.to_numpy(), want[k])
        assert actx.k_report(i)[1]["rebuilds"] >= 1
        t.free()


def test_device_reads_with_bad_offsets(kh, actx):
    """Reads on the device whose offsets decrease are refused before any
    read is reordered."""
    import torch
    reads = synth.config(1, scale=0.05)
    dev = kh.DeviceReads.from_host(reads)
    off = dev.offsets.clone()
    off[5] = off[7]  # read 5 would end before it starts
    bad = kh.DeviceReads(dev.seq, dev.qual, off)
    with pytest.raises(kh.KHError):
        actx.count(bad, 21, use_bloom=True)
    torch.cuda.synchronize()
    # the context still works
    assert_same_table(actx.count(dev, 21, use_bloom=True).to_numpy(), oracle.count(reads, 21))
