"""Read localisation on the GPU against the localisation oracle: the order
of the reads (grouped by the contig of their first contig k-mer) must equal
the oracle's exactly, the gathered reads must be the input's reads in that
order, and tables counted from them must equal the input's (the change is a
pure performance variant)."""
import numpy as np
import pytest

import brute
import oracle
import synth
from brute import assert_same_table
from test_traverse_pins import _random_genome

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lctx(kh):
    c = kh.Context(0)
    yield c
    c.close()


def _check_order(kh, lctx, reads, k, **count_kw):
    t = lctx.count(reads, k, **count_kw)
    c = lctx.traverse(t)
    seqs = c.to_python()["seqs"]
    want = oracle.localize(reads, seqs, k)
    got_host = lctx.localize_order(t, c, reads)
    dev = kh.DeviceReads.from_host(reads)
    got_dev = lctx.localize_order(t, c, dev).cpu().numpy()
    print("k=%d reads=%d contigs=%d" % (k, reads.n_reads, len(seqs)), flush=True)
    np.testing.assert_array_equal(got_host, want)
    np.testing.assert_array_equal(got_dev, want)
    c.free()
    t.free()
    return want, dev


@pytest.mark.parametrize("k", [21, 33, 77, 99])
def test_small_workload(kh, lctx, k):
    _check_order(kh, lctx, synth.config(1, scale=0.3), k)


def test_metagenome_sample(kh, lctx):
    _check_order(kh, lctx, synth.config(2, scale=0.01), 21, use_bloom=True)


@pytest.mark.parametrize("seed", range(10))
def test_random_reads(kh, lctx, seed):
    rng = np.random.default_rng(7100 + seed)
    k = int(rng.choice([5, 11, 21, 33, 55]))
    g = _random_genome(rng, int(rng.integers(100, 800)))
    pairs = []
    for _ in range(int(rng.integers(1, 300))):
        a = int(rng.integers(0, max(1, len(g) - 10)))
        s = list(g[a:a + int(rng.integers(1, 120))])
        for i in range(len(s)):
            u = rng.random()
            if u < 0.01:
                s[i] = "N"
            elif u < 0.03:
                s[i] = "ACGT"[int(rng.integers(0, 4))]
            elif u < 0.05:
                s[i] = s[i].lower()
        s = "".join(s)
        pairs.append((brute.revcomp(s.upper()) if rng.random() < 0.4 else s, "I" * len(s)))
    _check_order(kh, lctx, synth.Reads.from_strings(pairs), k, min_count=1)


def test_gathered_reads_and_unchanged_tables(kh, lctx):
    import torch
    reads = synth.config(2, scale=0.01)
    order, dev = _check_order(kh, lctx, reads, 21, use_bloom=True)
    moved = lctx.gather_reads(dev, torch.from_numpy(order).to(dev.seq.device))
    strings = reads.strings()
    want = synth.Reads.from_strings([strings[i] for i in order])
    np.testing.assert_array_equal(moved.offsets.cpu().numpy(), want.offsets)
    np.testing.assert_array_equal(moved.seq.cpu().numpy(), want.seq)
    np.testing.assert_array_equal(moved.qual.cpu().numpy(), want.qual)
    for k in (33, 55):
        got = lctx.count(moved, k, use_bloom=True).to_numpy()
        assert_same_table(got, oracle.count(reads, k))


def test_errors(kh, lctx):
    import torch
    reads = synth.config(1, scale=0.05)
    dev = kh.DeviceReads.from_host(reads)
    n = reads.n_reads
    bad = torch.arange(n, dtype=torch.int64, device=dev.seq.device)
    bad[0] = n  # out of range
    with pytest.raises(kh.KHError):
        lctx.gather_reads(dev, bad)
    dup = torch.arange(n, dtype=torch.int64, device=dev.seq.device)
    dup[1] = 0  # read 0 twice, read 1 never: lengths differ in this data set
    if reads.offsets[1] - reads.offsets[0] != reads.offsets[2] - reads.offsets[1]:
        with pytest.raises(kh.KHError):
            lctx.gather_reads(dev, dup)
    t = lctx.count(reads, 21)
    t2 = lctx.count(reads, 21)
    c = lctx.traverse(t)
    with pytest.raises(kh.KHError):
        lctx.localize_order(t2, c, reads)  # contigs walked from another table
    empty = synth.Reads.from_strings([])
    assert len(lctx.localize_order(t, c, empty)) == 0
    c.free()
    t.free()
    t2.free()


def test_full_size_permutation_and_tables(kh, lctx):
    """The 10M-read metagenome localised by its k = 21 contigs: the order is
    a permutation, and the k = 33 table of the localised reads equals the
    input's byte for byte."""
    import time
    import torch
    reads = synth.config(2)
    dev = kh.DeviceReads.from_host(reads)
    t = lctx.count(dev, 21, use_bloom=True)
    c = lctx.traverse(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    order = lctx.localize_order(t, c, dev)
    moved = lctx.gather_reads(dev, order)
    torch.cuda.synchronize()
    print("localise + gather %.1f ms" % ((time.perf_counter() - t0) * 1e3), flush=True)
    c.free()
    t.free()
    srt, _ = torch.sort(order)
    assert torch.equal(srt, torch.arange(reads.n_reads, dtype=torch.int64, device=order.device))
    del srt
    a = lctx.count(dev, 33, use_bloom=True)
    b = lctx.count(moved, 33, use_bloom=True)
    ta, tb = a.to_numpy(), b.to_numpy()
    a.free()
    b.free()
    assert_same_table(ta, tb)
