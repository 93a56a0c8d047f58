"""Pins for the CPU oracle (no GPU needed).

The oracle is checked against things other than itself: a hand-worked table,
an independent brute force on random and exhaustive tiny inputs, closed-form
window totals, extension totals counted a different way, reverse-complement
and order invariance, special cases with known answers, hand-built classifier
vectors and the generator's ground-truth genome.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
import synth
from brute import assert_same_table, key_words, revcomp, table as brute_table

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _reads(pairs):
    return synth.Reads.from_strings(pairs)


def _random_case(rng, k):
    glen = int(rng.integers(50, 301))
    genome = "".join(rng.choice(list("ACGT"), size=glen))
    pairs = []
    for _ in range(int(rng.integers(5, 51))):
        L = int(rng.integers(5, 41))
        a = int(rng.integers(0, max(1, glen - L)))
        s = list(genome[a:a + L])
        if rng.random() < 0.5:
            s = list(revcomp("".join(s)))
        for j in range(len(s)):
            u = rng.random()
            if u < 0.03:
                s[j] = "N"
            elif u < 0.06:
                s[j] = s[j].lower()
            elif u < 0.09:
                s[j] = "ACGT"[int(rng.integers(0, 4))]
        q = "".join(chr(33 + int(x)) for x in rng.integers(0, 42, size=len(s)))
        pairs.append(("".join(s), q))
    return pairs


# --------------------------------------------------------------- golden ----

def _load_golden(name):
    reads, rows, totals = [], [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "READ":
                reads.append((t[1], t[2]))
            elif t[0] == "ROW":
                rows.append((t[1], int(t[2]), [int(x) for x in t[3:11]], t[11]))
            elif t[0] == "TOTAL":
                totals = {t[i]: int(t[i + 1]) for i in range(1, len(t), 2)}
    k = len(rows[0][0])
    return reads, rows, totals, k


@pytest.mark.parametrize("min_count", [1, 2])
def test_golden_hand_k3(min_count):
    reads, rows, totals, k = _load_golden("hand_k3.txt")
    o = oracle.count(_reads(reads), k, min_count=min_count)
    want = [r for r in rows if r[1] >= min_count]
    assert o["n_rows"] == len(want)
    for i, (text, cnt, ext, code) in enumerate(want):
        assert list(o["keys"][i]) == key_words(text)
        assert int(o["counts"][i]) == cnt
        assert list(o["ext"][i]) == ext
        assert o["codes"][i].tobytes().decode() == code
    assert o["n_windows"] == totals["windows"]
    assert o["n_distinct"] == totals["distinct"]
    assert o["sum_left"] == totals["left"]
    assert o["sum_right"] == totals["right"]


# ---------------------------------------------------------- brute force ----

@pytest.mark.parametrize("seed", range(24))
def test_bruteforce_random(seed):
    rng = np.random.default_rng(9000 + seed)
    k = [1, 3, 5, 7, 21, 2, 4][seed % 7]
    kw = dict(min_count=int(rng.integers(1, 4)),
              qual_cutoff=int(rng.choice([0, 20, 30])),
              t_min_ext=int(rng.integers(0, 4)), t_base=int(rng.integers(0, 3)),
              err_ppm=int(rng.choice([0, 5000, 300000])))
    pairs = _random_case(rng, k)
    assert_same_table(oracle.count(_reads(pairs), k, **kw),
                      brute_table(pairs, k, **kw))


@pytest.mark.parametrize("k", [1, 3, 5])
def test_bruteforce_exhaustive(k):
    rng = np.random.default_rng(77 + k)
    pairs = []
    for L in range(1, 7):
        for t in itertools.product("ACGTN", repeat=L):
            q = "".join(chr(33 + int(x)) for x in rng.integers(10, 40, size=L))
            pairs.append(("".join(t), q))
    for mc in (1, 2, 5):
        assert_same_table(oracle.count(_reads(pairs), k, min_count=mc),
                          brute_table(pairs, k, min_count=mc))


def test_bruteforce_catches_planted_mistakes():
    """The comparison is sensitive: brute-force variants with a plausible
    mistake (no complement on the strand swap; left/right not swapped;
    quality cutoff exclusive) all disagree with the oracle."""
    rng = np.random.default_rng(5)
    pairs = _random_case(rng, 5)
    o = oracle.count(_reads(pairs), 5, min_count=1)
    good = brute_table(pairs, 5, min_count=1)
    assert_same_table(o, good)

    import brute

    def variant(swap_comp=True, swap_sides=True, cutoff_inclusive=True):
        from collections import Counter, defaultdict
        count, left, right = Counter(), defaultdict(lambda: [0] * 4), defaultdict(lambda: [0] * 4)
        for s, q in pairs:
            s = "".join(ch.upper() if ch in "acgt" else ch for ch in s)
            for i in range(len(s) - 4):
                w = s[i:i + 5]
                if not set(w) <= set("ACGT"):
                    continue
                def hq(j):
                    ph = ord(q[j]) - 33
                    return ph >= 20 if cutoff_inclusive else ph > 20
                fl = s[i - 1] if i > 0 and s[i - 1] in "ACGT" and hq(i - 1) else ""
                fr = s[i + 5] if i + 5 < len(s) and s[i + 5] in "ACGT" and hq(i + 5) else ""
                rc = revcomp(w)
                if rc < w:
                    a, b = (fr, fl) if swap_sides else (fl, fr)
                    if swap_comp:
                        a, b = revcomp(a), revcomp(b)
                    key, L, R = rc, a, b
                else:
                    key, L, R = w, fl, fr
                count[key] += 1
                if L:
                    left[key]["ACGT".index(L)] += 1
                if R:
                    right[key]["ACGT".index(R)] += 1
        return sorted((key, count[key], tuple(left[key]), tuple(right[key])) for key in count)

    ref = variant()
    assert ref == sorted((t, int(c), tuple(e[:4]), tuple(e[4:]))
                         for t, c, e in zip(good["text"], good["counts"], good["ext"].tolist()))
    assert variant(swap_comp=False) != ref
    assert variant(swap_sides=False) != ref
    # the exclusive cutoff only differs if some neighbour has Phred exactly 20
    pairs.append(("ACGTACGTAC", "IIIII5IIII"))  # '5' = Phred 20
    ref2 = variant()
    assert variant(cutoff_inclusive=False) != ref2
    del brute


# ---------------------------------------------------------- closed forms ----

def _acgt_runs(s):
    run, out = 0, []
    for ch in s:
        if ch in "ACGTacgt":
            run += 1
        else:
            out.append(run)
            run = 0
    out.append(run)
    return out


def test_closed_form_windows_workload1():
    r = synth.config(1)
    for k in (21, 33, 55):
        o = oracle.count(r, k)
        assert o["n_windows"] == r.n_reads * (151 - k)
    assert oracle.count(r, 21)["n_windows"] == 866_710


@pytest.mark.parametrize("seed", range(6))
def test_closed_form_windows_with_n(seed):
    rng = np.random.default_rng(300 + seed)
    k = [3, 5, 7][seed % 3]
    pairs = _random_case(rng, k)
    want = sum(max(0, run - k + 1) for s, _ in pairs for run in _acgt_runs(s))
    assert oracle.count(_reads(pairs), k, min_count=1)["n_windows"] == want


@pytest.mark.parametrize("seed", range(6))
def test_extension_totals(seed):
    """Sum of all extension tallies = number of (window, side) pairs whose
    neighbour exists, is a base and has Phred >= cutoff; per row, each side's
    tallies sum to at most the count."""
    rng = np.random.default_rng(400 + seed)
    k = [3, 5, 21][seed % 3]
    pairs = _random_case(rng, k)
    n_side = 0
    for s, q in pairs:
        good = [ch in "ACGTacgt" for ch in s]
        hq = [good[j] and ord(q[j]) - 33 >= 20 for j in range(len(s))]
        for i in range(len(s) - k + 1):
            if all(good[i:i + k]):
                n_side += (i > 0 and hq[i - 1]) + (i + k < len(s) and hq[i + k])
    o = oracle.count(_reads(pairs), k, min_count=1)
    assert o["sum_left"] + o["sum_right"] == n_side
    assert np.all(o["ext"][:, :4].sum(1) <= o["counts"])
    assert np.all(o["ext"][:, 4:].sum(1) <= o["counts"])


# ------------------------------------------------------------ invariants ----

def _rc_reads(r):
    comp = np.zeros(256, np.uint8)
    comp[:] = np.arange(256, dtype=np.uint8)
    for a, b in zip(b"ACGTacgt", b"TGCAtgca"):
        comp[a] = b
    seq = np.empty_like(r.seq)
    qual = np.empty_like(r.qual)
    for i in range(r.n_reads):
        a, b = int(r.offsets[i]), int(r.offsets[i + 1])
        seq[a:b] = comp[r.seq[a:b]][::-1]
        qual[a:b] = r.qual[a:b][::-1]
    return synth.Reads(seq, qual, r.offsets.copy())


@pytest.mark.parametrize("k", [1, 5, 21, 33, 77])
def test_rc_invariance(k):
    r = synth.config(1, scale=0.3)
    rng = np.random.default_rng(k)
    r.seq[rng.integers(0, r.n_bases, size=50)] = ord("N")
    assert_same_table(oracle.count(r, k), oracle.count(_rc_reads(r), k))


def test_order_invariance():
    r = synth.config(1, scale=0.3)
    perm = np.random.default_rng(3).permutation(r.n_reads)
    pairs = r.strings()
    shuffled = _reads([pairs[i] for i in perm])
    assert_same_table(oracle.count(r, 21), oracle.count(shuffled, 21))


# --------------------------------------------------------- special cases ----

@pytest.mark.parametrize("base", ["A", "T"])
def test_homopolymer(base):
    n, k = 40, 21
    o = oracle.count(_reads([(base * n, "I" * n)]), k, min_count=1)
    assert o["n_rows"] == 1
    assert list(o["keys"][0]) == key_words("A" * k)
    assert int(o["counts"][0]) == n - k + 1
    assert list(o["ext"][0]) == [n - k, 0, 0, 0, n - k, 0, 0, 0]
    assert o["codes"][0].tobytes() == b"AA"


def test_cutoff_extremes():
    r = synth.config(1, scale=0.2)
    raw = oracle.count(r, 21, qual_cutoff=0, min_count=1)
    pairs = r.strings()
    # cutoff 0: tallies are the raw neighbour counts
    n_side = sum((len(s) - 21) * 2 for s, _ in pairs)  # no N in workload 1
    assert raw["sum_left"] + raw["sum_right"] == n_side
    none = oracle.count(r, 21, qual_cutoff=94, min_count=1)
    assert none["sum_left"] == none["sum_right"] == 0
    assert np.all(none["codes"] == ord("X"))


def test_min_count_one_keeps_everything():
    r = synth.config(1, scale=0.1)
    o = oracle.count(r, 21, min_count=1)
    assert o["n_rows"] == o["n_distinct"]
    assert int(o["counts"].sum()) == o["n_windows"]


def test_distinct_kmers_single_read_empty():
    s = "ACGTTGCAAGGCTTACCGATAGCTAGGATCCAGTAAC"
    o = oracle.count(_reads([(s, "I" * len(s))]), 11, min_count=2)
    assert o["n_rows"] == 0 and o["n_windows"] == len(s) - 10


def test_k1_two_keys():
    s = "AACGTTTGCAGN"
    o = oracle.count(_reads([(s, "I" * len(s))]), 1, min_count=1)
    na = s.count("A") + s.count("T")
    nc = s.count("C") + s.count("G")
    assert [list(x) for x in o["keys"]] == [[0], [1]]
    assert list(o["counts"]) == [na, nc]


def test_read_shorter_than_k_and_k_equals_length():
    s = "ACGTACGTAC"
    o = oracle.count(_reads([(s[:5], "IIIII")]), 7, min_count=1)
    assert o["n_rows"] == 0 and o["n_windows"] == 0
    o = oracle.count(_reads([(s, "I" * 10)]), 9, min_count=1)
    assert o["n_windows"] == 2
    o = oracle.count(_reads([(s[:9], "I" * 9)]), 9, min_count=1)
    assert o["n_windows"] == 1 and o["sum_left"] == 0 and o["sum_right"] == 0


def test_empty_input():
    r = synth.Reads(np.zeros(0, np.uint8), np.zeros(0, np.uint8),
                    np.zeros(1, np.int64))
    o = oracle.count(r, 21)
    assert o["n_rows"] == 0 and o["n_windows"] == 0


# ------------------------------------------------------------ classifier ----

@pytest.mark.parametrize("c,depth,kw,want", [
    ([0, 0, 0, 0], 5, {}, "X"),                       # no extension
    ([1, 0, 0, 0], 5, {}, "X"),                       # m = t_min_ext - 1
    ([2, 0, 0, 0], 5, {}, "A"),                       # m = t_min_ext
    ([0, 0, 3, 3], 6, {}, "F"),                       # tie for the maximum
    ([5, 1, 0, 0], 6, {}, "A"),                       # alt = t_base exactly
    ([5, 1, 1, 0], 7, {}, "F"),                       # alt = t_base + 1
    ([0, 300, 2, 0], 400, {}, "C"),                   # e*d = 2.0, alt = 2
    ([0, 300, 3, 0], 400, {}, "F"),                   # e*d = 2.0, alt = 3
    ([0, 0, 0, 1000], 1200, {}, "T"),                 # high depth, no alt
    ([0, 0, 2, 1000], 1200, {"err_ppm": 0}, "F"),     # global t_hq = t_base
    ([0, 0, 1, 1000], 1200, {"err_ppm": 0}, "T"),
    ([0, 0, 0, 1], 1, {"t_min_ext": 1}, "T"),
    ([0, 0, 0, 0], 1, {"t_min_ext": 0}, "F"),         # all tied at zero
    ([7, 0, 0, 0], 7, {"t_base": 0}, "A"),
    ([7, 1, 0, 0], 8, {"t_base": 0}, "F"),
])
def test_classifier_cases(c, depth, kw, want):
    assert oracle.classify_side(c, depth, **kw) == want


# ---------------------------------------------------- generator ground truth

def test_generator_ground_truth_workload1():
    """At 20x coverage nearly every genomic 21-mer is kept; the codes of
    genomic k-mers away from the genome ends are mostly unique letters."""
    seed = synth.BASE_SEED + 100
    g, off = synth.genomes(seed, [50_000], [0.5])
    genome = g.tobytes().decode()
    r = synth.config(1)
    o = oracle.count(r, 21)
    kept = {tuple(x) for x in o["keys"].tolist()}
    kmers = set()
    for i in range(len(genome) - 20):
        w = genome[i:i + 21]
        rc = revcomp(w)
        kmers.add(tuple(key_words(min(w, rc))))
    frac = len(kmers & kept) / len(kmers)
    assert frac >= 0.999, frac
    codes = o["codes"]
    unique = np.isin(codes, np.frombuffer(b"ACGT", np.uint8)).all(1).mean()
    assert unique > 0.99


# ----------------------------------------------------- shards and queries ----

def _np_mix64(z):
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xbf58476d1ce4e5b9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94d049bb133111eb)
    return z ^ (z >> np.uint64(31))


def shard_np(keys, S):
    h = np.zeros(keys.shape[0], np.uint64)
    for w in range(keys.shape[1]):
        h = _np_mix64(h ^ keys[:, w])
    return h % np.uint64(S)


@pytest.mark.parametrize("k", [21, 55])
def test_shards_partition_table(k):
    r = synth.config(1, scale=0.3)
    full = oracle.count(r, k)
    S = 5
    sh = shard_np(full["keys"], S)
    for i in range(3):
        assert oracle.shard_of(full["keys"][i], S) == int(sh[i])
    total = 0
    for s in range(S):
        part = oracle.count_shard(r, k, S, s)
        m = sh == s
        sub = {f: full[f][m] for f in ("keys", "counts", "ext", "codes")}
        sub["n_rows"] = int(m.sum())
        assert_same_table(part, sub, totals=False)
        total += part["n_windows"]
    assert total == full["n_windows"]


def test_count_keys_matches_table():
    r = synth.config(1, scale=0.3)
    full = oracle.count(r, 33, min_count=1)
    idx = np.random.default_rng(1).choice(full["n_rows"], 40, replace=False)
    q = full["keys"][idx]
    q = np.concatenate([q, np.array([[0, 0]], np.uint64)])  # AAA...A: unseen
    counts, ext = oracle.count_keys(r, 33, q)
    np.testing.assert_array_equal(counts[:-1], full["counts"][idx])
    np.testing.assert_array_equal(ext[:-1], full["ext"][idx])
    assert counts[-1] == 0
