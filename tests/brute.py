"""Brute-force k-mer tables for tiny inputs (pin for the C oracle).

Written independently of ``oracle/oracle.c``: Python string slicing,
``str.translate`` for the reverse complement, ``collections.Counter`` for the
tallies and Python big integers for the 2-bit key words.  It follows the same
definition (paper Section II-B/II-C plus the readings listed in the design
notes) and is only meant for inputs of a few thousand windows.
"""
from collections import Counter, defaultdict

import numpy as np

_COMP = str.maketrans("ACGT", "TGCA")
_DIGITS = str.maketrans("ACGT", "0123")


def revcomp(s: str) -> str:
    return s.translate(_COMP)[::-1]


def key_words(kmer: str) -> list:
    k = len(kmer)
    W = (k + 31) // 32
    v = int(kmer.translate(_DIGITS), 4)
    return [(v >> (64 * (W - 1 - i))) & ((1 << 64) - 1) for i in range(W)]


def side_letter(c, depth, t_min_ext=2, t_base=1, err_ppm=5000) -> str:
    m = max(c)
    if m < t_min_ext:
        return "X"
    if sum(1 for x in c if x == m) > 1:
        return "F"
    alt = sum(c) - m
    ok = alt * 10**6 <= max(t_base * 10**6, err_ppm * depth)
    return "ACGT"[c.index(m)] if ok else "F"


def table(pairs, k, min_count=2, qual_offset=33, qual_cutoff=20, t_min_ext=2,
          t_base=1, err_ppm=5000):
    """pairs: [(seq, qual)] strings.  Returns dict with the same fields as the
    oracle wrapper (keys/counts/ext/codes arrays sorted by key + totals)."""
    count = Counter()
    left = defaultdict(lambda: [0, 0, 0, 0])
    right = defaultdict(lambda: [0, 0, 0, 0])
    ok = set("ACGT")
    for s, q in pairs:
        s = "".join(ch.upper() if ch in "acgt" else ch for ch in s)
        for i in range(len(s) - k + 1):
            w = s[i:i + k]
            if not set(w) <= ok:
                continue
            fl = s[i - 1] if i > 0 and s[i - 1] in ok and \
                ord(q[i - 1]) - qual_offset >= qual_cutoff else ""
            fr = s[i + k] if i + k < len(s) and s[i + k] in ok and \
                ord(q[i + k]) - qual_offset >= qual_cutoff else ""
            rc = revcomp(w)
            if rc < w:
                key, L, R = rc, revcomp(fr), revcomp(fl)
            else:
                key, L, R = w, fl, fr
            count[key] += 1
            if L:
                left[key]["ACGT".index(L)] += 1
            if R:
                right[key]["ACGT".index(R)] += 1
    keys = sorted(kk for kk, c in count.items() if c >= min_count)
    W = (k + 31) // 32
    n = len(keys)
    out = dict(k=k, W=W, n_rows=n,
               keys=np.array([key_words(x) for x in keys], dtype=np.uint64).reshape(n, W),
               counts=np.array([count[x] for x in keys], dtype=np.uint32),
               ext=np.array([left[x] + right[x] for x in keys], dtype=np.uint32).reshape(n, 8),
               codes=np.array([[ord(side_letter(left[x], count[x], t_min_ext, t_base, err_ppm)),
                                ord(side_letter(right[x], count[x], t_min_ext, t_base, err_ppm))]
                               for x in keys], dtype=np.uint8).reshape(n, 2),
               n_windows=sum(count.values()), n_distinct=len(count),
               sum_left=sum(sum(v) for v in left.values()),
               sum_right=sum(sum(v) for v in right.values()),
               text=keys)
    return out


def assert_same_table(a: dict, b: dict, totals: bool = True):
    """Row-for-row equality of two tables (and the pre-threshold totals)."""
    assert a["n_rows"] == b["n_rows"], (a["n_rows"], b["n_rows"])
    np.testing.assert_array_equal(a["keys"], b["keys"])
    np.testing.assert_array_equal(a["counts"], b["counts"])
    np.testing.assert_array_equal(a["ext"], b["ext"])
    np.testing.assert_array_equal(a["codes"], b["codes"])
    if totals:
        for f in ("n_windows", "sum_left", "sum_right"):
            if f in a and f in b and a[f] is not None and b[f] is not None:
                assert a[f] == b[f], (f, a[f], b[f])


# ------------------------------------------------------------ contigs ----

_COMP_CODE = str.maketrans("ACGT", "TGCA")  # F and X stay


def key_text(words, k: int) -> str:
    v = 0
    for w in words:
        v = (v << 64) | int(w)
    return "".join("ACGT"[(v >> (2 * (k - 1 - j))) & 3] for j in range(k))


def contigs(t: dict, mutual: bool = True) -> list:
    """Contigs of a table by brute force: every mutual unique edge between
    k-mers is collected from a dict of all rows, components are joined with a
    union-find, and each component is written from any end that has no left
    edge (or, for a cycle, from its smallest k-mer).  Returns [(sequence,
    n_kmers, depth, is_cycle)] ordered by each contig's smallest k-mer."""
    k = t["k"]
    rows = {}
    for i in range(t["n_rows"]):
        rows[key_text(t["keys"][i], k)] = (chr(int(t["codes"][i][0])),
                                           chr(int(t["codes"][i][1])),
                                           int(t["counts"][i]))

    def canon(s):
        r = revcomp(s)
        return (s, True) if s <= r else (r, False)

    def codes(s):  # (left, right) of a k-mer read in this orientation
        c, fwd = canon(s)
        L, R, _ = rows[c]
        return (L, R) if fwd else (R.translate(_COMP_CODE), L.translate(_COMP_CODE))

    def right_of(s):
        R = codes(s)[1]
        if R not in "ACGT":
            return None
        n = s[1:] + R
        c = canon(n)[0]
        if c not in rows or c == canon(s)[0] or (mutual and codes(n)[0] != s[0]):
            return None
        return n

    def left_of(s):
        L = codes(s)[0]
        if L not in "ACGT":
            return None
        p = L + s[:-1]
        c = canon(p)[0]
        if c not in rows or c == canon(s)[0] or (mutual and codes(p)[1] != s[-1]):
            return None
        return p

    parent = {s: s for s in rows}

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for s in rows:
        for o in (s, revcomp(s)):
            n = right_of(o)
            if n is not None:
                a, b = find(s), find(canon(n)[0])
                if a != b:
                    parent[a] = b
    comps = defaultdict(list)
    for s in rows:
        comps[find(s)].append(s)
    out = []
    for nodes in comps.values():
        start = None
        for s in sorted(nodes):
            for o in (s, revcomp(s)):
                if left_of(o) is None:
                    start = o
                    break
            if start is not None:
                break
        cycle = start is None
        if cycle:
            start = min(nodes)
        seq, cur, seen = start, start, 1
        while True:
            n = right_of(cur)
            if n is None or (cycle and canon(n)[0] == start):
                break
            seq += n[-1]
            cur = n
            seen += 1
            assert seen <= len(nodes)
        assert seen == len(nodes)
        if not cycle:
            seq = min(seq, revcomp(seq))
        out.append((min(nodes), seq, len(nodes), sum(rows[s][2] for s in nodes), cycle))
    out.sort()
    return [x[1:] for x in out]


def merge(t: dict, contig_list: list, override: bool = False) -> dict:
    """Table rows merged with every k-mer of the contigs, by brute force:
    rows and contig k-mers in Python dicts keyed by canonical text.  With
    override=True (a planted mistake) contig k-mers replace existing rows."""
    k, W = t["k"], t["W"]
    rows = {}
    for i in range(t["n_rows"]):
        rows[key_text(t["keys"][i], k)] = (int(t["counts"][i]), [int(x) for x in t["ext"][i]],
                                           chr(int(t["codes"][i][0])) + chr(int(t["codes"][i][1])))
    sides = defaultdict(lambda: [set(), set(), False, False])  # left bases, right bases, no-left, no-right
    ok = set("ACGT")
    for c in contig_list:
        c = c.upper()
        for p in range(len(c) - k + 1):
            w = c[p:p + k]
            if not set(w) <= ok:
                continue
            fl = c[p - 1] if p > 0 and c[p - 1] in ok else ""
            fr = c[p + k] if p + k < len(c) and c[p + k] in ok else ""
            rc = revcomp(w)
            key, L, R = (rc, revcomp(fr), revcomp(fl)) if rc < w else (w, fl, fr)
            s = sides[key]
            if L:
                s[0].add(L)
            else:
                s[2] = True
            if R:
                s[1].add(R)
            else:
                s[3] = True

    def code(bases, none):
        if not bases:
            return "X"
        return next(iter(bases)) if len(bases) == 1 and not none else "F"

    for key, (lb, rb, ln, rn) in sides.items():
        if key in rows and not override:
            continue
        rows[key] = (0, [0] * 8, code(lb, ln) + code(rb, rn))
    keys = sorted(rows)
    n = len(keys)
    return dict(k=k, W=W, n_rows=n,
                keys=np.array([key_words(x) for x in keys], dtype=np.uint64).reshape(n, W),
                counts=np.array([rows[x][0] for x in keys], dtype=np.uint32),
                ext=np.array([rows[x][1] for x in keys], dtype=np.uint32).reshape(n, 8),
                codes=np.array([[ord(rows[x][2][0]), ord(rows[x][2][1])] for x in keys],
                               dtype=np.uint8).reshape(n, 2))


def prune_neighbours(contig_list: list, k: int) -> list:
    """For every contig, the set of other contigs holding a k-mer that
    overlaps its first k-mer by k-1 bases on the left or its last k-mer by
    k-1 bases on the right (any base, either strand)."""
    owner = {}
    for ci, c in enumerate(contig_list):
        for p in range(len(c) - k + 1):
            w = c[p:p + k]
            owner[min(w, revcomp(w))] = ci
    out = []
    for ci, c in enumerate(contig_list):
        near = set()
        for b in "ACGT":
            for w in (b + c[:k - 1], c[len(c) - k + 1:] + b):
                j = owner.get(min(w, revcomp(w)))
                if j is not None and j != ci:
                    near.add(j)
        out.append(near)
    return out


def prune(contig_list: list, k: int, depth, alpha: float, beta: float,
          synchronous: bool = True, pooled: bool = True):
    """Iterative pruning by brute force over Python sets and floats.
    Returns (removed_at, sweeps).  synchronous=False (removals take effect at
    once, in contig order) and pooled=False (the neighbourhood's depth as the
    mean of the neighbours' mean depths) are planted mistakes."""
    n = len(contig_list)
    near = prune_neighbours(contig_list, k)
    nk = [len(c) - k + 1 for c in contig_list]
    mean = [float(int(depth[i])) / float(nk[i]) for i in range(n)]
    alive = [True] * n
    removed = [-1] * n
    g = 1.0 + alpha
    tau, sweeps = 1.0, 0
    while True:
        left = [mean[i] for i in range(n) if alive[i]]
        if not left or not tau < max(left):
            break
        state = list(alive)
        for i in range(n):
            seen = state if synchronous else alive
            if not alive[i] or len(contig_list[i]) > 2 * k:
                continue
            nb = [j for j in near[i] if seen[j]]
            if not nb:
                continue
            if pooled:
                nd = float(sum(int(depth[j]) for j in nb)) / float(sum(nk[j] for j in nb))
            else:
                nd = sum(mean[j] for j in nb) / len(nb)
            if mean[i] <= min(tau, beta * nd):
                alive[i] = False
                removed[i] = sweeps
        sweeps += 1
        tau = tau * g
    return removed, sweeps


def localize(read_strings: list, contig_list: list, k: int) -> list:
    """Read order by brute force: each read's first window found among the
    contigs' k-mers (a dict from canonical text to the first contig holding
    it) names its contig; reads sorted by that, stably, unanchored last."""
    owner = {}
    for ci, c in enumerate(contig_list):
        c = c.upper()
        for p in range(len(c) - k + 1):
            w = c[p:p + k]
            if set(w) <= set("ACGT"):
                owner.setdefault(min(w, revcomp(w)), ci)
    keys = []
    for r in read_strings:
        r = r.upper()
        key = len(contig_list)
        for p in range(len(r) - k + 1):
            w = r[p:p + k]
            if set(w) <= set("ACGT") and min(w, revcomp(w)) in owner:
                key = owner[min(w, revcomp(w))]
                break
        keys.append(key)
    return sorted(range(len(read_strings)), key=lambda i: keys[i])
