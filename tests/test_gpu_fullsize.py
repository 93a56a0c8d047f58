"""Parity at full size: the 10M-read metagenome at k = 21..99 in the batched
call bench.py times.  The oracle cannot build whole tables of this size, so:

* properties that hold at any size are checked on every row (window total,
  strict key order, threshold, tallies bounded by the count, codes equal to
  the classification of each row's own tallies);
* sampled rows are recounted exactly by the oracle (every window of every
  read is scanned for the sampled keys);
* sampled windows taken straight from the reads are looked up: a k-mer the
  oracle counts at least twice must be a row with the oracle's record, one
  it counts once must be absent.
"""
import numpy as np
import pytest

import oracle
import synth
from brute import key_words, revcomp, side_letter

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


def _find(keys, q):
    """Row index of key q in the sorted key matrix, or -1."""
    lo, hi = 0, keys.shape[0]
    qt = tuple(int(x) for x in q)
    while lo < hi:
        mid = (lo + hi) // 2
        if tuple(int(x) for x in keys[mid]) < qt:
            lo = mid + 1
        else:
            hi = mid
    if lo < keys.shape[0] and tuple(int(x) for x in keys[lo]) == qt:
        return lo
    return -1


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


@pytest.mark.parametrize("k", KS)
def test_fullsize_sampled_exact(full, k):
    reads, tabs = full
    t = tabs[k]
    rng = np.random.default_rng(100 + k)
    # sampled rows
    rows = rng.choice(t["n_rows"], 24, replace=False)
    q_rows = t["keys"][rows]
    # sampled windows straight from the reads
    q_win = []
    for _ in range(24):
        r = int(rng.integers(0, reads.n_reads))
        a = int(reads.offsets[r])
        i = int(rng.integers(0, 151 - k))
        w = reads.seq[a + i:a + i + k].tobytes().decode()
        q_win.append(key_words(min(w, revcomp(w))))
    q = np.concatenate([q_rows, np.array(q_win, np.uint64).reshape(-1, t["W"])])
    counts, ext = oracle.count_keys(reads, k, q)
    for j in range(len(rows)):
        assert int(counts[j]) == int(t["counts"][rows[j]])
        assert ext[j].tolist() == t["ext"][rows[j]].tolist()
    for j in range(len(q_win)):
        c = int(counts[len(rows) + j])
        assert c >= 1  # the window is in the reads
        idx = _find(t["keys"], q[len(rows) + j])
        if c >= 2:
            assert idx >= 0
            assert int(t["counts"][idx]) == c
            assert t["ext"][idx].tolist() == ext[len(rows) + j].tolist()
        else:
            assert idx < 0


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
