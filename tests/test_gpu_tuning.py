"""Tuning parameters (windows per lane, tiles per block, load factor, Bloom
bits) and the autotuner: every setting must give the oracle's table."""
import numpy as np
import pytest

import oracle
import synth
from brute import assert_same_table

pytestmark = pytest.mark.gpu

SHAPES = [  # (count_lanes, bloom_lanes, tiles_per_block)
    (1, 1, 1), (2, 2, 3), (4, 1, 8), (1, 4, 1024), (2, 4, 2), (0, 4, 4),
]


@pytest.fixture(scope="module")
def w1():
    return synth.config(1, scale=0.3)


@pytest.fixture
def tctx(kh):
    """The single-table path, whose launch shapes these tests vary."""
    c = kh.Context(0)
    c.set_tuning(partitioned=0)
    yield c
    c.close()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bloom", [False, True])
def test_launch_shapes_same_table(kh, tctx, w1, shape, bloom):
    cl, bl, tpb = shape
    tctx.set_tuning(count_lanes=cl, bloom_lanes=bl, tiles_per_block=tpb)
    ks = [21, 33, 77, 99]
    want = {k: oracle.count(w1, k) for k in ks}
    for k in ks:  # single-k path
        assert_same_table(tctx.count(w1, k, use_bloom=bloom).to_numpy(), want[k])
    tabs = tctx.count_multi_k(w1, ks, use_bloom=bloom)  # batched path
    for k, t in zip(ks, tabs):
        assert_same_table(t.to_numpy(), want[k])


@pytest.mark.parametrize("shape", [(1, 1, 4), (2, 2, 1)])
def test_heavy_and_rebuild_under_shapes(kh, tctx, monkeypatch, shape):
    cl, bl, tpb = shape
    tctx.set_tuning(count_lanes=cl, bloom_lanes=bl, tiles_per_block=tpb)
    pairs = [("A" * 100, "I" * 100)] * 900 + synth.config(1, scale=0.05).strings()
    reads = synth.Reads.from_strings(pairs)
    ks = [21, 55]
    monkeypatch.setenv("KMERHIP_FORCE_CAPACITY", "500")
    tabs = tctx.count_multi_k(reads, ks, use_bloom=True)
    for k, t in zip(ks, tabs):
        got = t.to_numpy()
        assert_same_table(got, oracle.count(reads, k))
    assert int(tabs[0].to_numpy()["counts"].max()) > 4096


@pytest.mark.parametrize("lf,bits", [(0.3, 2), (0.9, 1), (0.05, 64)])
def test_load_factor_and_bloom_bits(kh, tctx, w1, lf, bits):
    tctx.set_tuning(load_factor=lf, bloom_bits=bits)
    got = tctx.count(w1, 33, use_bloom=True).to_numpy()
    assert_same_table(got, oracle.count(w1, 33))
    # the parameters of the call override the context's tuning
    got = tctx.count(w1, 33, use_bloom=True, load_factor=0.5, bloom_bits=3).to_numpy()
    assert_same_table(got, oracle.count(w1, 33))


def test_set_tuning_errors(kh, tctx):
    before = tctx.tuning()
    bad = [dict(load_factor=0.95), dict(load_factor=0.0), dict(bloom_bits=0),
           dict(bloom_bits=65), dict(count_lanes=3), dict(bloom_lanes=8),
           dict(tiles_per_block=0), dict(tiles_per_block=1025), dict(partitioned=2),
           dict(tails_overlap=2)]
    for b in bad:
        with pytest.raises(kh.KHError) as e:
            tctx.set_tuning(**b)
        assert e.value.code == kh.KH_EINVAL
        assert tctx.tuning() == before
    with pytest.raises(kh.KHError) as e:
        tctx.count(synth.config(1, scale=0.01), 21, bloom_bits=65)
    assert e.value.code == kh.KH_EINVAL


def test_autotune(kh, tctx, w1):
    ks = [21, 33, 55]
    tuned, rep = tctx.autotune(w1, ks, use_bloom=True)
    print("tuned", tuned, rep, flush=True)
    assert tctx.tuning() == tuned
    # the owner-partitioned count, when it wins, ends the search: the other
    # fields shape the single-table path only
    assert rep["trials"] >= (2 if tuned["partitioned"] else 10)
    assert rep["best_ms"] <= rep["start_ms"]
    assert tuned["count_lanes"] in (0, 1, 2, 4) and tuned["bloom_lanes"] in (1, 2, 4)
    tabs = tctx.count_multi_k(w1, ks, use_bloom=True)
    for k, t in zip(ks, tabs):
        assert_same_table(t.to_numpy(), oracle.count(w1, k))
    with pytest.raises(kh.KHError) as e:
        tctx.autotune(w1, ks, reps=0)
    assert e.value.code == kh.KH_EINVAL


def test_autotune_cached(kh, tctx, w1, tmp_path):
    """The stored choice: the first call tunes and appends a line, the second
    (a fresh context) takes it without trials; tables stay the oracle's."""
    cache = str(tmp_path / "tuning.txt")
    ks = [21, 33]
    dev = kh.DeviceReads.from_host(w1)
    t1, r1, hit1 = tctx.autotune_cached(dev, ks, cache, use_bloom=True)
    assert not hit1 and r1["trials"] > 0
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and "ks=21,33" in lines[0] and "bloom=1" in lines[0]
    assert "reads=%d" % w1.n_reads in lines[0]
    other = kh.Context(0)
    try:
        t2, r2, hit2 = other.autotune_cached(dev, ks, cache, use_bloom=True)
        assert hit2 and r2["trials"] == 0
        assert t2 == t1 and other.tuning() == t1
        want = {k: oracle.count(w1, k) for k in ks}
        for k, t in zip(ks, other.count_multi_k(dev, ks, use_bloom=True)):
            assert_same_table(t.to_numpy(), want[k])
        # another case (Bloom off) is not the stored one
        _, _, hit3 = other.autotune_cached(dev, ks, cache, use_bloom=False)
        assert not hit3 and len(open(cache).read().splitlines()) == 2
    finally:
        other.close()


@pytest.mark.parametrize("overlap", [0, 1])
def test_tails_schedule_same_table(kh, tctx, w1, overlap):
    """The batched call's tails beside the later counting passes or after
    the last one: the same tables."""
    tctx.set_tuning(tails_overlap=overlap)
    ks = [21, 33, 55, 77, 99]
    want = {k: oracle.count(w1, k) for k in ks}
    for k, t in zip(ks, tctx.count_multi_k(w1, ks, use_bloom=True)):
        assert_same_table(t.to_numpy(), want[k])
