"""Contigs and their pruning at full size: the 10M-read metagenome's k = 21
table (1.7e8 rows, Bloom screen on).  The oracles cannot walk or prune a
graph of this size in a test, so:

* the multiset of k-mers spelled by all contigs equals the table's rows
  exactly (every row lies in exactly one contig, every contig k-mer is a
  row) -- checked vectorised over all contigs;
* lengths, k-mer numbers and depth totals agree with the table;
* sampled contigs are valid maximal walks: consecutive k-mers are joined by
  mutual unique codes, the ends have no mutual edge beyond them, a path is
  written in its smaller orientation, and its depth is the sum of its
  k-mers' counts;
* pruning (Algorithm 2): the sweep count follows from the threshold
  schedule and the running largest depth, no contig over 2k bases goes, and
  for a sample of short contigs every sweep's decision is recomputed from
  its neighbours (found from the sorted rows) and the sweeps that removed
  them.
"""
import numpy as np
import pytest

import brute
import synth

pytestmark = pytest.mark.gpu

K = 21
_CODE = np.full(256, 255, np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _CODE[_c] = _i


@pytest.fixture(scope="module")
def full():
    import paper_1809_07014_amd as kh
    reads = synth.config(2)
    ctx = kh.Context(0)
    dev = kh.DeviceReads.from_host(reads)
    t = ctx.count(dev, K, use_bloom=True)
    c = ctx.traverse(t)
    info = c.info()
    kept, rep, removed = ctx.prune(t, c, removed_at=True)
    rep["kept"] = kept.info()["n_contigs"]
    kept.free()
    tab = t.to_numpy()
    ct = c.to_numpy()
    ct["removed_at"], ct["prune"] = removed, rep
    c.free()
    t.free()
    ctx.close()
    print("rows=%d contigs=%d bases=%d rounds=%d cycle_kmers=%d" % (
        tab["n_rows"], info["n_contigs"], info["total_bases"], info["rounds"],
        info["cycle_kmers"]), flush=True)
    return tab, ct


def _kmer_values(codes, starts):
    """Forward and reverse-complement 2-bit values of the k-mers at starts
    (codes: the contigs' bases as 0..3)."""
    v = np.zeros(len(starts), np.uint64)
    r = np.zeros(len(starts), np.uint64)
    for j in range(K):
        v = (v << np.uint64(2)) | codes[starts + j].astype(np.uint64)
        r = (r << np.uint64(2)) | (3 - codes[starts + K - 1 - j]).astype(np.uint64)
    return v, r


def test_every_row_in_exactly_one_contig(full):
    tab, ct = full
    off, seq = ct["offsets"], ct["seq"]
    lens = np.diff(off)
    assert np.all(lens == K + ct["n_kmers"] - 1)
    assert int(ct["n_kmers"].sum()) == tab["n_rows"]
    assert int(ct["depth"].sum()) == int(tab["counts"].sum(dtype=np.uint64))
    codes = _CODE[seq]
    assert np.all(codes < 4)
    # start of every k-mer in every contig
    nk = ct["n_kmers"]
    starts = np.repeat(off[:-1], nk) + (np.arange(int(nk.sum())) -
                                        np.repeat(np.cumsum(nk) - nk, nk))
    v = np.zeros(len(starts), np.uint64)
    r = np.zeros(len(starts), np.uint64)
    for j in range(K):
        v = (v << np.uint64(2)) | codes[starts + j].astype(np.uint64)
        r = (r << np.uint64(2)) | (3 - codes[starts + K - 1 - j]).astype(np.uint64)
    canon = np.minimum(v, r)
    canon.sort()
    np.testing.assert_array_equal(canon, tab["keys"][:, 0])


def test_sampled_contigs_are_maximal_walks(full):
    tab, ct = full
    keys = tab["keys"][:, 0]

    def row(s):
        c = min(s, brute.revcomp(s))
        v = np.uint64(int(c.translate(str.maketrans("ACGT", "0123")), 4))
        i = int(np.searchsorted(keys, v))
        return i if i < len(keys) and keys[i] == v else -1

    comp = str.maketrans("ACGTFX", "TGCAFX")

    def codes(s):
        i = row(s)
        L, R = chr(tab["codes"][i][0]), chr(tab["codes"][i][1])
        return (L, R) if s <= brute.revcomp(s) else (R.translate(comp), L.translate(comp))

    def right_of(s):
        R = codes(s)[1]
        if R not in "ACGT":
            return None
        n = s[1:] + R
        if row(n) < 0 or row(n) == row(s) or codes(n)[0] != s[0]:
            return None
        return n

    def left_of(s):
        L = codes(s)[0]
        if L not in "ACGT":
            return None
        p = L + s[:-1]
        if row(p) < 0 or row(p) == row(s) or codes(p)[1] != s[-1]:
            return None
        return p

    rng = np.random.default_rng(3)
    off = ct["offsets"]
    raw = ct["seq"]
    picks = rng.choice(ct["n_contigs"], 150, replace=False)
    big = np.argsort(ct["n_kmers"])[-10:]  # the longest contigs too
    for ci in list(picks) + list(big):
        s = raw[off[ci]:off[ci + 1]].tobytes().decode()
        n = int(ct["n_kmers"][ci])
        for p in list(range(min(n, 200) - 1)) + list(range(max(0, n - 200), n - 1)):
            assert right_of(s[p:p + K]) == s[p + 1:p + 1 + K]
        if not ct["cycle"][ci]:
            assert left_of(s[:K]) is None and right_of(s[-K:]) is None
            assert s <= brute.revcomp(s)
        if n <= 400:
            assert int(ct["depth"][ci]) == sum(int(tab["counts"][row(s[p:p + K])])
                                               for p in range(n))


def test_pruning_at_full_size(full):
    tab, ct = full
    keys = tab["keys"][:, 0]
    removed, rep = ct["removed_at"], ct["prune"]
    alpha, beta = 0.1, 0.2  # the library's defaults
    off, nk, depth = ct["offsets"], ct["n_kmers"], ct["depth"]
    lens = np.diff(off)
    mean = depth.astype(np.float64) / nk.astype(np.float64)
    sweeps = rep["sweeps"]
    print("sweeps=%d removed=%d kept=%d" % (sweeps, rep["removed"], rep["kept"]), flush=True)
    assert rep["removed"] == int((removed >= 0).sum()) > 0
    assert rep["kept"] == int((removed < 0).sum())
    assert np.all(removed[lens > 2 * K] == -1)
    assert removed.max() < sweeps
    taus, tau = [], 1.0
    for _ in range(sweeps + 1):
        taus.append(tau)
        tau = tau * (1.0 + alpha)
    for s in range(sweeps):  # each sweep ran because tau was below the maximum
        assert taus[s] < mean[(removed < 0) | (removed >= s)].max()
    assert not taus[sweeps] < mean[removed < 0].max()
    # contig of every row: sort all contig k-mers by canonical value
    starts = np.repeat(off[:-1], nk) + (np.arange(int(nk.sum())) -
                                        np.repeat(np.cumsum(nk) - nk, nk))
    codes = _CODE[ct["seq"]]
    v, r = _kmer_values(codes, starts)
    order = np.argsort(np.minimum(v, r))  # keys are distinct
    row_contig = np.repeat(np.arange(len(nk)), nk)[order]
    del v, r, order, starts
    print("row -> contig map built", flush=True)

    def holder(vals):
        i = np.searchsorted(keys, vals)
        i = np.minimum(i, len(keys) - 1)
        return np.where(keys[i] == vals, row_contig[i], -1)

    rng = np.random.default_rng(11)
    short = np.flatnonzero(lens <= 2 * K)
    gone = np.flatnonzero(removed >= 0)
    sample = np.unique(np.concatenate([rng.choice(short, 1500, replace=False),
                                       rng.choice(gone, min(1500, len(gone)), replace=False)]))
    mask = np.uint64((1 << (2 * K)) - 1)
    for n_done, c in enumerate(sample):
        if n_done % 500 == 0:
            print("checked %d of %d sampled contigs" % (n_done, len(sample)), flush=True)
        fv, _ = _kmer_values(codes, np.array([off[c]]))
        lv, _ = _kmer_values(codes, np.array([off[c + 1] - K]))
        cand = []
        for b in range(4):
            bb = np.uint64(b)
            left = (fv >> np.uint64(2)) | (bb << np.uint64(2 * K - 2))  # b + first[0..k-1)
            right = ((lv << np.uint64(2)) & mask) | bb                  # last[1..k) + b
            for x in (left, right):
                rc = np.zeros(1, np.uint64)
                y = x.copy()
                for _ in range(K):
                    rc = (rc << np.uint64(2)) | (np.uint64(3) - (y & np.uint64(3)))
                    y >>= np.uint64(2)
                cand.append(min(int(x[0]), int(rc[0])))
        near = set(int(j) for j in holder(np.array(cand, np.uint64)) if j >= 0 and j != c)
        last = removed[c] if removed[c] >= 0 else sweeps - 1
        for s in range(last + 1):
            nb = [j for j in near if removed[j] < 0 or removed[j] >= s]
            go = False
            if nb:
                nd = float(sum(int(depth[j]) for j in nb)) / float(sum(int(nk[j]) for j in nb))
                go = mean[c] <= min(taus[s], beta * nd)
            assert go == (s == removed[c]), (c, s, removed[c])
