"""Host reads uploaded in chunks by the batched and the single-k call, each
chunk's Bloom pass overlapping the next chunk's copy.  KMERHIP_STREAM_CHUNK shrinks the chunks
so that small read sets take this path: tables must equal the oracle's,
for chunk sizes that split reads and tiles anywhere, with reads of mixed
length and ambiguous bases, and when the tables do not fit at once and the
call counts the k one after another."""
import numpy as np
import pytest

import brute
import oracle
import synth
from brute import assert_same_table
from test_traverse_pins import _random_genome

pytestmark = pytest.mark.gpu

KS = [21, 33, 55, 77, 99]


@pytest.fixture(scope="module")
def sctx(kh):
    """Single-table path: the one whose Bloom pass overlaps the upload (the
    owner-partitioned count finishes the upload before routing)."""
    c = kh.Context(0)
    c.set_tuning(partitioned=0)
    yield c
    c.close()


def test_owner_path_after_streamed_pack(kh, monkeypatch):
    monkeypatch.setenv("KMERHIP_STREAM_CHUNK", "5000")
    reads = synth.config(1)
    c = kh.Context(0)
    try:
        for k, t in zip(KS, c.count_multi_k(reads, KS, use_bloom=True)):
            assert_same_table(t.to_numpy(), oracle.count(reads, k))
            t.free()
        t = c.count(reads, 55, use_bloom=True)
        assert_same_table(t.to_numpy(), oracle.count(reads, 55))
        t.free()
    finally:
        c.close()


@pytest.mark.parametrize("chunk", [1024, 5000, 65536])
def test_small_workload_streamed(sctx, monkeypatch, chunk):
    monkeypatch.setenv("KMERHIP_STREAM_CHUNK", str(chunk))
    reads = synth.config(1)
    tabs = sctx.count_multi_k(reads, KS, use_bloom=True)
    for k, t in zip(KS, tabs):
        assert_same_table(t.to_numpy(), oracle.count(reads, k))
        t.free()


@pytest.mark.parametrize("k", [21, 55, 99])
def test_single_k_streamed(sctx, monkeypatch, k):
    """kh_count streams host reads the same way through its Bloom pass."""
    monkeypatch.setenv("KMERHIP_STREAM_CHUNK", "7000")
    reads = synth.config(1)
    t = sctx.count(reads, k, use_bloom=True)
    assert_same_table(t.to_numpy(), oracle.count(reads, k))
    t.free()
    t = sctx.count(reads, k, use_bloom=True, owner_shards=3, owner=1)  # a key-space part
    want = oracle.count_shard(reads, k, 3, 1)
    got = t.to_numpy()
    assert_same_table(got, want, totals=False)
    assert got["n_windows"] == want["n_windows"]
    t.free()


def test_mixed_reads_streamed(sctx, monkeypatch):
    monkeypatch.setenv("KMERHIP_STREAM_CHUNK", "3000")
    rng = np.random.default_rng(77)
    g = _random_genome(rng, 20_000)
    pairs = []
    for _ in range(2500):
        n = int(rng.integers(0, 400))
        a = int(rng.integers(0, len(g) - n))
        s = list(g[a:a + n])
        for i in range(n):
            if rng.random() < 0.005:
                s[i] = "N"
        s = "".join(s)
        q = "".join(chr(33 + int(x)) for x in rng.integers(2, 42, size=n))
        pairs.append((brute.revcomp(s) if rng.random() < 0.5 else s, q))
    reads = synth.Reads.from_strings(pairs)
    ks = [21, 33, 127]
    tabs = sctx.count_multi_k(reads, ks, use_bloom=True, min_count=2)
    for k, t in zip(ks, tabs):
        assert_same_table(t.to_numpy(), oracle.count(reads, k, min_count=2))
        t.free()


def test_streamed_under_budgets(kh, monkeypatch):
    """Shrinking budgets: the batched call either fits, falls back to one k
    at a time (which must first finish the upload), or reports KH_ENOMEM."""
    monkeypatch.setenv("KMERHIP_STREAM_CHUNK", "4096")
    reads = synth.config(1)
    want = {k: oracle.count(reads, k) for k in KS}
    fitted = []
    for mb in range(64, 8, -3):
        c = kh.Context(0, hbm_budget=mb << 20)
        try:
            tabs = c.count_multi_k(reads, KS, use_bloom=True)
        except kh.KHError as e:
            assert e.code == kh.KH_ENOMEM
            c.close()
            break
        for k, t in zip(KS, tabs):
            assert_same_table(t.to_numpy(), want[k])
            t.free()
        fitted.append(mb)
        c.close()
    print("budgets that fit (MB):", fitted, flush=True)
    assert fitted
