"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Integer work, so every comparison is exact (keys, counts, all eight
extension tallies, both code letters, and the window total).
"""
import os

import numpy as np
import pytest

import oracle
import synth
from brute import assert_same_table, key_words, revcomp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(kh):
    c = kh.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def single(kh):
    """A context on the single-table path (one device hash table per k)."""
    c = kh.Context(0)
    c.set_tuning(partitioned=0)
    yield c
    c.close()


@pytest.fixture(params=["owner", "single"])
def anyctx(request, ctx, single):
    """Both counting paths: owner-partitioned (the default) and single-table."""
    return ctx if request.param == "owner" else single


@pytest.fixture(scope="module")
def w1():
    return synth.config(1)


def _check(ctx, kh, reads, k, device=True, **kw):
    src = kh.DeviceReads.from_host(reads) if device else reads
    got = ctx.count(src, k, **kw).to_numpy()
    okw = {x: kw[x] for x in ("min_count", "qual_cutoff", "t_min_ext", "t_base",
                              "err_ppm") if x in kw}
    want = oracle.count(reads, k, **okw)
    print("k=%d rows=%d windows=%d" % (k, want["n_rows"], want["n_windows"]), flush=True)
    assert_same_table(got, want)
    assert got["n_windows"] == want["n_windows"]
    return got


def test_workload1_k21_plain(anyctx, kh, w1):
    got = _check(anyctx, kh, w1, 21)
    assert got["n_windows"] == 866_710


def test_workload1_k21_bloom(anyctx, kh, w1):
    _check(anyctx, kh, w1, 21, use_bloom=True)


@pytest.mark.parametrize("k", [1, 3, 5, 11, 31, 33, 35, 55, 61, 63, 65, 67, 77, 95,
                               97, 99, 123, 125, 127])
def test_every_key_width(anyctx, kh, k):
    """Every key width and every record / LDS-chunk width of the owner path
    (k = 35 and 67 are the only odd k of two of them)."""
    r = synth.config(1, scale=0.15)
    _check(anyctx, kh, r, k, min_count=1 if k < 15 else 2)


@pytest.mark.parametrize("seed", range(12))
def test_random_small_sets(anyctx, kh, seed):
    """Variable read lengths, N and lowercase bases, random qualities."""
    rng = np.random.default_rng(5000 + seed)
    k = [1, 3, 5, 7, 21, 33][seed % 6]
    glen = 400
    genome = "".join(rng.choice(list("ACGT"), size=glen))
    pairs = []
    for _ in range(300):
        L = int(rng.integers(0, 90))
        a = int(rng.integers(0, glen - L + 1))
        s = list(genome[a:a + L])
        if rng.random() < 0.5:
            s = list(revcomp("".join(s)))
        for j in range(len(s)):
            u = rng.random()
            if u < 0.02:
                s[j] = "N"
            elif u < 0.04:
                s[j] = s[j].lower()
        q = "".join(chr(33 + int(x)) for x in rng.integers(0, 42, size=len(s)))
        pairs.append(("".join(s), q))
    reads = synth.Reads.from_strings(pairs)
    kw = dict(min_count=int(rng.integers(1, 4)),
              qual_cutoff=int(rng.choice([0, 20, 30])),
              t_min_ext=int(rng.integers(0, 4)), t_base=int(rng.integers(0, 3)),
              err_ppm=int(rng.choice([0, 5000, 300000])))
    _check(anyctx, kh, reads, k, device=bool(seed % 2), **kw)


def test_host_and_device_reads_agree(ctx, kh, w1):
    a = ctx.count(w1, 21).to_numpy()
    b = ctx.count(kh.DeviceReads.from_host(w1), 21).to_numpy()
    assert_same_table(a, b)


@pytest.mark.parametrize("bits", [1, 2, 8, 32])
def test_bloom_invariance(anyctx, kh, bits):
    """Bloom on (any size, even saturated) == Bloom off."""
    r = synth.config(2, scale=0.002)
    off = anyctx.count(r, 21).to_numpy()
    on = anyctx.count(r, 21, use_bloom=True, bloom_bits=bits).to_numpy()
    assert_same_table(on, off)
    assert on["n_windows"] == off["n_windows"]


def test_rebuild_after_probe_limit(ctx, kh, w1, monkeypatch):
    """A table forced far too small is rebuilt until every key fits; the
    result is unchanged."""
    r = synth.config(1, scale=0.05)
    want = oracle.count(r, 21)
    monkeypatch.setenv("KMERHIP_FORCE_CAPACITY", "300")
    got = ctx.count(r, 21).to_numpy()
    assert ctx.stats()["rebuilds"] >= 1
    assert_same_table(got, want)


def test_order_and_rc_invariance(anyctx, kh):
    r = synth.config(1, scale=0.3)
    base = anyctx.count(r, 33).to_numpy()
    perm = np.random.default_rng(1).permutation(r.n_reads)
    pairs = r.strings()
    shuf = synth.Reads.from_strings([pairs[i] for i in perm])
    assert_same_table(anyctx.count(shuf, 33).to_numpy(), base)
    rc = synth.Reads.from_strings([(revcomp(s), q[::-1]) for s, q in pairs])
    assert_same_table(anyctx.count(rc, 33).to_numpy(), base)


@pytest.mark.parametrize("ks,bloom", [([21, 33, 55, 77, 99], True),
                                      ([21, 33, 55, 77, 99], False),
                                      ([25, 21, 23, 27, 31, 45, 63], True),
                                      ([99, 21], True)])
@pytest.mark.parametrize("path", ["owner", "single"])
def test_multi_k_matches_single(ctx, single, kh, ks, bloom, path):
    """The multi-k call equals one single-k call per k of the other path.
    Single-table path: the batched call (fused Bloom launches,
    graph-captured counting passes, tails on a second stream), on every
    replay of the captured graph, with eager work between replays."""
    multi, other = (ctx, single) if path == "owner" else (single, ctx)
    r = synth.config(1, scale=0.3)
    want = {k: other.count(r, k, use_bloom=bloom).to_numpy() for k in ks}
    dev = kh.DeviceReads.from_host(r)
    for rep in range(3):
        tabs = multi.count_multi_k(dev, ks, use_bloom=bloom)
        for k, t in zip(ks, tabs):
            got = t.to_numpy()
            assert_same_table(got, want[k])
            assert got["n_windows"] == want[k]["n_windows"]
        multi.count(synth.config(1, scale=0.05), 21)  # eager work between replays


def test_graphed_passes_equal_eager(single, kh, monkeypatch):
    """The counting passes replayed as one graph record their start and end
    events as external nodes (the side stream's tails wait on the end
    events from outside the graph): every k's counting time is positive
    and the tables equal those of the same call with eager launches."""
    r = synth.config(1, scale=0.3)
    dev = kh.DeviceReads.from_host(r)
    ks = [21, 33, 55, 77, 99]
    single.set_timing(True)
    try:
        graphed, g_ms = [], []
        for rep in range(2):
            tabs = single.count_multi_k(dev, ks, use_bloom=True)
            assert single.last_graphed()
            g_ms.append([single.k_report(i)[0]["count"] for i in range(len(ks))])
            assert min(g_ms[-1]) > 0
            graphed.append([t.to_numpy() for t in tabs])
            for t in tabs:
                t.free()
        monkeypatch.setenv("KMERHIP_NO_GRAPH", "1")
        tabs = single.count_multi_k(dev, ks, use_bloom=True)
        assert not single.last_graphed()
        e_ms = [single.k_report(i)[0]["count"] for i in range(len(ks))]
        for i, t in enumerate(tabs):
            eager = t.to_numpy()
            t.free()
            assert e_ms[i] > 0
            for g in graphed:
                assert_same_table(g[i], eager)
        # each pass's events bracket that pass only: an end event recorded
        # late (after later passes) would add their times to this one's
        print("graphed ms", g_ms, "eager ms", e_ms, flush=True)
        assert sum(g_ms[-1]) <= 2 * sum(e_ms) + 2.0
    finally:
        single.set_timing(False)


def test_multi_k_rebuild_and_heavy(ctx, kh, monkeypatch):
    """Rebuild after a probe runs out and the heavy-hitter recount inside the
    batched multi-k call."""
    pairs = [("A" * 100, "I" * 100)] * 900 + synth.config(1, scale=0.05).strings()
    reads = synth.Reads.from_strings(pairs)
    ks = [21, 33, 55]
    want = {k: oracle.count(reads, k) for k in ks}
    monkeypatch.setenv("KMERHIP_FORCE_CAPACITY", "500")
    tabs = ctx.count_multi_k(reads, ks, use_bloom=True)
    for i, (k, t) in enumerate(zip(ks, tabs)):
        assert_same_table(t.to_numpy(), want[k])
        assert ctx.k_report(i)[1]["rebuilds"] >= 1


def test_edge_inputs(anyctx, kh):
    empty = synth.Reads(np.zeros(0, np.uint8), np.zeros(0, np.uint8),
                        np.zeros(1, np.int64))
    t = anyctx.count(empty, 21).to_numpy()
    assert t["n_rows"] == 0 and t["n_windows"] == 0
    short = synth.Reads.from_strings([("ACGT", "IIII"), ("", ""), ("NNNNNNNNNNNN", "I" * 12)])
    t = anyctx.count(short, 5, min_count=1).to_numpy()
    assert t["n_rows"] == 0 and t["n_windows"] == 0
    one = synth.Reads.from_strings([("ACGTACGTAC", "IIIIIIIIII")])
    _check(anyctx, kh, one, 9, min_count=1)
    _check(anyctx, kh, one, 1, min_count=1)
    homo = synth.Reads.from_strings([("A" * 150, "I" * 150), ("T" * 150, "I" * 150)])
    t = _check(anyctx, kh, homo, 21)
    assert list(t["keys"][0]) == key_words("A" * 21)


@pytest.mark.parametrize("bloom", [False, True])
def test_heavy_hitters_exact(anyctx, kh, bloom):
    """k-mers seen more than 65535 times (beyond the 16-bit tallies of the
    main table) get exact tallies from the heavy-hitter recount."""
    rng = np.random.default_rng(11)
    pairs = [("A" * 100, "I" * 100)] * 900 + [("ACGT" * 30, "I" * 120)] * 1400
    for _ in range(200):
        s = "".join(rng.choice(list("ACGT"), size=100))
        q = "".join(chr(33 + int(x)) for x in rng.integers(2, 42, size=100))
        pairs.append(("A" * 30 + s, "I" * 30 + q))
    reads = synth.Reads.from_strings(pairs)
    got = _check(anyctx, kh, reads, 21, use_bloom=bloom)
    assert got["counts"].max() > 65535


@pytest.mark.parametrize("extra", [16, 17, 18, 19])
def test_heavy_threshold_boundary(anyctx, kh, extra):
    """Counts just below, at and above the packed-tally limit (4096):
    48 * 80 + 3 * 79 + (extra + 1) = 4094 .. 4097 occurrences of A^21."""
    pairs = [("A" * 100, "I" * 100)] * 48 + [("A" * (21 + extra), "I" * (21 + extra))]
    pairs += [("C" + "A" * 99, "5" + "I" * 99)] * 3  # one low-quality left base
    reads = synth.Reads.from_strings(pairs)
    got = _check(anyctx, kh, reads, 21)
    assert int(got["counts"][0]) == 4078 + extra


@pytest.mark.parametrize("n_tails,long_run", [(20, False), (200, True)])
@pytest.mark.parametrize("path", ["owner", "single"])
def test_equal_key_prefixes(ctx, single, kh, n_tails, long_run, path):
    """Many 55-mers sharing their top 32 bases.  Single-table path: short
    runs of equal sort prefixes are ordered by the full key; a long run
    falls back to the full-key sort.  Owner path: all of them land in one
    owner, whose bucket sort orders them by the full key.  Either way the
    rows match the oracle."""
    c = ctx if path == "owner" else single
    rng = np.random.default_rng(21 + n_tails)
    head = "AAAAC" + "".join(rng.choice(list("ACGT"), size=27))
    pairs = []
    for _ in range(n_tails):
        tail = "".join(rng.choice(list("ACG"), size=28))
        pairs += [(head + tail, "I" * 60)] * 2
    reads = synth.Reads.from_strings(pairs)
    _check(c, kh, reads, 55)
    if path == "single":
        assert c.stats()["full_key_sort"] == int(long_run)


def test_parameter_errors(ctx, kh, w1):
    for k in (0, 2, 22, 128, 129):
        with pytest.raises(kh.KHError) as e:
            ctx.count(w1, k)
        assert e.value.code == kh.KH_EINVAL
    with pytest.raises(kh.KHError):
        ctx.count(w1, 21, min_count=0)
    with pytest.raises(kh.KHError):
        ctx.count(w1, 21, min_count=4097)
    with pytest.raises(kh.KHError):
        ctx.count(w1, 21, min_count=1, use_bloom=True)
    bad = synth.Reads(w1.seq, w1.qual, w1.offsets.copy())
    bad.offsets[5] = bad.offsets[7]
    with pytest.raises(kh.KHError) as e:
        ctx.count(bad, 21)
    assert e.value.code == kh.KH_EINVAL
    # decreasing offsets detected on the device
    with pytest.raises(kh.KHError) as e:
        ctx.count(kh.DeviceReads.from_host(bad), 21)
    assert e.value.code == kh.KH_EINVAL


def test_budget_exceeded(kh, w1):
    small = kh.Context(0, hbm_budget=1 << 20)
    with pytest.raises(kh.KHError) as e:
        small.count(w1, 21)
    assert e.value.code == kh.KH_ENOMEM
    small.close()


def test_table_outlives_context(kh, w1):
    c = kh.Context(0)
    t = c.count(w1, 21)
    c.close()
    assert t.info()["n_rows"] == 0
    t.free()


def test_memory_kept_across_contexts(kh, w1):
    """A destroyed context's blocks serve the next context on the device, and
    give the same result; release_cached hands them back to the driver."""
    want = oracle.count(w1, 27)
    for _ in range(2):
        c = kh.Context(0)
        assert_same_table(c.count(w1, 27).to_numpy(), want)
        c.close()
    kh.release_cached(0)
    c = kh.Context(0)
    assert_same_table(c.count(w1, 27).to_numpy(), want)
    c.close()
    kh.release_cached(0)
    with pytest.raises(kh.KHError) as e:
        kh.release_cached(4096)
    assert e.value.code == kh.KH_EINVAL


def test_trim_keeps_live_tables(kh, w1):
    """kh_trim returns cached blocks only: a live table keeps its rows."""
    c = kh.Context(0)
    t = c.count(w1, 21)
    c.count(w1, 33).free()  # leaves cached blocks behind
    c.trim()
    assert_same_table(t.to_numpy(), oracle.count(w1, 21))
    assert_same_table(c.count(w1, 33).to_numpy(), oracle.count(w1, 33))
    t.free()
    c.close()
