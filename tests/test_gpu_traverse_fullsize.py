"""Contigs at full size: the 10M-read metagenome's k = 21 table (1.7e8
rows, Bloom screen on).  The oracle cannot walk a graph of this size, so:

* the multiset of k-mers spelled by all contigs equals the table's rows
  exactly (every row lies in exactly one contig, every contig k-mer is a
  row) -- checked vectorised over all contigs;
* lengths, k-mer numbers and depth totals agree with the table;
* sampled contigs are valid maximal walks: consecutive k-mers are joined by
  mutual unique codes, the ends have no mutual edge beyond them, a path is
  written in its smaller orientation, and its depth is the sum of its
  k-mers' counts.
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
    tab = t.to_numpy()
    ct = c.to_numpy()
    c.free()
    t.free()
    ctx.close()
    print("rows=%d contigs=%d bases=%d rounds=%d cycle_kmers=%d" % (
        tab["n_rows"], info["n_contigs"], info["total_bases"], info["rounds"],
        info["cycle_kmers"]), flush=True)
    return tab, ct


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
