"""Parity at full size: the 10M-read metagenome at k = 21..99 in the batched
call bench.py times.  The oracle cannot build whole tables of this size, so:

* properties that hold at any size are checked on every row (window total,
  strict key order, threshold, tallies bounded by the count, codes equal to
  the classification of each row's own tallies);
* one complete part of the k-mer space per k is compared row for row with
  the oracle: the oracle counts every window of every read and keeps the
  k-mers of shard s of 64 (its own implementation of the partition
  function), and the GPU export, filtered to the same shard, must equal it
  exactly -- keys, counts, all eight tallies and both code letters.  A row
  missing from the GPU table, a row it should not have (a k-mer seen once
  that passed the Bloom screen), or any wrong field fails.
"""
import time

import numpy as np
import pytest

import oracle
import synth
from brute import assert_same_table, side_letter
from test_oracle_pins import shard_np

pytestmark = pytest.mark.gpu

KS = (21, 33, 55, 77, 99)


@pytest.fixture(scope="module")
def full():
    import paper_1809_07014_amd as kh
    reads = synth.config(2)
    ctx = kh.Context(0)
    dev = kh.DeviceReads.from_host(reads)
    tabs = ctx.count_multi_k(dev, KS, use_bloom=True)
    out = {k: t.to_numpy() for k, t in zip(KS, tabs)}
    for t in tabs:
        t.free()
    ctx.close()
    return reads, out


@pytest.mark.parametrize("k", KS)
def test_fullsize_properties(full, k):
    reads, tabs = full
    t = tabs[k]
    print("k=%d rows=%d windows=%d" % (k, t["n_rows"], t["n_windows"]), flush=True)
    assert t["n_windows"] == reads.n_reads * (151 - k)  # 150 bp reads, no N
    keys = t["keys"]
    # strictly increasing keys (lexicographic over words)
    if keys.shape[1] == 1:
        assert np.all(keys[1:, 0] > keys[:-1, 0])
    else:
        a, b = keys[:-1], keys[1:]
        gt = np.zeros(len(a), bool)
        eq = np.ones(len(a), bool)
        for w in range(keys.shape[1]):
            gt |= eq & (b[:, w] > a[:, w])
            eq &= b[:, w] == a[:, w]
        assert np.all(gt)
    assert np.all(t["counts"] >= 2)
    assert np.all(t["ext"][:, :4].sum(1) <= t["counts"])
    assert np.all(t["ext"][:, 4:].sum(1) <= t["counts"])
    # codes are the classification of each row's own tallies (sampled)
    rng = np.random.default_rng(k)
    for i in rng.choice(t["n_rows"], 2000, replace=False):
        c, e = int(t["counts"][i]), t["ext"][i].tolist()
        want = side_letter(e[:4], c) + side_letter(e[4:], c)
        assert t["codes"][i].tobytes().decode() == want


SHARDS = 64


@pytest.mark.parametrize("k", KS)
def test_fullsize_shard_exact(full, k):
    """A complete shard of the table, row for row against the oracle."""
    reads, tabs = full
    t = tabs[k]
    s = (7 * k) % SHARDS
    t0 = time.time()
    want = oracle.count_shard(reads, k, SHARDS, s)
    print("k=%d oracle shard %d of %d: %d rows in %.1f s" %
          (k, s, SHARDS, want["n_rows"], time.time() - t0), flush=True)
    sel = shard_np(t["keys"], SHARDS) == s
    got = dict(k=k, W=t["W"], n_rows=int(sel.sum()), keys=t["keys"][sel],
               counts=t["counts"][sel], ext=t["ext"][sel], codes=t["codes"][sel])
    assert want["n_rows"] > 1000
    assert_same_table(got, want)


def test_fullsize_streamed_host_reads(full):
    """The same batched call from host reads, uploaded in 128 Mi-base chunks
    whose copies overlap the Bloom pass (bench.py's end-to-end leg), gives
    the same tables."""
    import paper_1809_07014_amd as kh
    reads, tabs = full
    ctx = kh.Context(0)
    got = ctx.count_multi_k(reads, KS, use_bloom=True)
    for k, t in zip(KS, got):
        g = t.to_numpy()
        t.free()
        assert g["n_windows"] == tabs[k]["n_windows"]
        for f in ("keys", "counts", "ext", "codes"):
            np.testing.assert_array_equal(g[f], tabs[k][f])
        del g
    ctx.close()
