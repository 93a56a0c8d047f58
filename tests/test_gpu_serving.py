"""Serving: continuous batching of read batches from many samples.

Each sample's tables after a mixed run (batches of several samples
interleaved, split into chunks that share launches, tables grown by rehash
while resident) must be bit-identical to counting the union of its batches
alone on the GPU, and to the CPU oracle's table of that union -- every
sample, every k.  The oracle's tables are computed in background threads
(the C oracle runs without the interpreter lock) while the GPU serves.
"""
import concurrent.futures as cf
import os
import time

import numpy as np
import pytest

import oracle
import synth
from brute import assert_same_table

pytestmark = pytest.mark.gpu

KS = (21, 33, 55)


def _samples(n, seed, reads_per_genome=1500, scale=0.002):
    specs = synth.serving_samples(n, reads_per_genome=reads_per_genome,
                                  scale=1.0, seed_offset=seed)
    out = []
    for spec in specs:
        spec = dict(spec)
        spec["lengths"] = np.maximum(2000, (spec["lengths"] * scale).astype(np.int64))
        out.append(synth.sample_reads(spec))
    return out


def _split(reads, rng, parts):
    cuts = sorted(rng.choice(np.arange(1, reads.n_reads), size=parts - 1, replace=False))
    bounds = [0] + [int(c) for c in cuts] + [reads.n_reads]
    return [reads.slice(bounds[i], bounds[i + 1]) for i in range(parts)]


def _union(batches):
    seq = np.concatenate([b.seq for b in batches])
    qual = np.concatenate([b.qual for b in batches])
    lens = np.concatenate([np.diff(b.offsets) for b in batches])
    off = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    return synth.Reads(seq, qual, off)


_POOL = None
_WANT = {}


def _oracle_tables(tag, samples):
    """Futures of the oracle's table of each sample at every k, keyed
    (sample index, k); started once per sample set."""
    global _POOL
    if _POOL is None:
        _POOL = cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1))
    if tag not in _WANT:
        _WANT[tag] = {(i, k): _POOL.submit(oracle.count, r, k)
                      for i, r in enumerate(samples) for k in KS}
    return _WANT[tag]


def _check_served(tabs, union, sample, want, i, ctx):
    """Served tables == the GPU alone on the union == the oracle's."""
    assert np.array_equal(union.seq, sample.seq)  # the batches cover the sample
    assert np.array_equal(union.offsets, sample.offsets)
    alone = ctx.count_multi_k(union, KS, use_bloom=False)
    for k, t, a in zip(KS, tabs, alone):
        got = t.to_numpy()
        assert_same_table(got, a.to_numpy())
        assert got["n_windows"] == a.info()["n_windows"]
        w = want[(i, k)].result()
        assert_same_table(got, w)
        assert got["n_windows"] == w["n_windows"]
        a.free()


@pytest.fixture(scope="module")
def ctx(kh):
    c = kh.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("plain", [False, True])
def test_mixed_equals_alone(kh, ctx, plain):
    rng = np.random.default_rng(7)
    samples = _samples(6, seed=11)
    want = _oracle_tables("mixed", samples)
    batches = {i: _split(r, rng, int(rng.integers(1, 5))) for i, r in enumerate(samples)}
    order = [(i, b) for i, bs in batches.items() for b in bs]
    rng.shuffle(order)
    srv = kh.Server(KS, max_active=3, chunk_reads=700, batch_bases=400_000,
                    plain=plain)
    tickets = []
    for i, b in order:  # Poisson-ish arrivals while earlier batches run
        tickets.append(srv.submit(100 + i, b))
        time.sleep(float(rng.exponential(0.002)))
    lat = [srv.wait(t) for t in tickets]
    assert all(x >= 0 for x in lat)
    st = srv.stats()
    print("stats", st, flush=True)
    assert st["completed"] == len(order)
    if not plain:
        assert st["max_active"] >= 2  # requests shared launches
        assert st["rehashes"] >= 1     # tables grew while resident
    for i in batches:
        tabs = srv.finalize(100 + i)
        _check_served(tabs, _union(batches[i]), samples[i], want, i, ctx)
    srv.close()


def test_overflow_replay(kh, ctx, monkeypatch):
    """Tables far too small: windows that find no slot are replayed into the
    grown table, and the result is still exact."""
    monkeypatch.setenv("KMERHIP_SERVER_TABLE_SLOTS", "512")
    rng = np.random.default_rng(21)
    samples = _samples(3, seed=5)
    want = _oracle_tables("overflow", samples)
    srv = kh.Server(KS, max_active=3, chunk_reads=500, batch_bases=300_000)
    monkeypatch.delenv("KMERHIP_SERVER_TABLE_SLOTS")
    batches = {i: _split(r, rng, 3) for i, r in enumerate(samples)}
    tickets = [srv.submit(7 + i, b) for i, bs in batches.items() for b in bs]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    print("stats", st, flush=True)
    assert st["replayed"] > 0 and st["rehashes"] >= 1
    for i in batches:
        tabs = srv.finalize(7 + i)
        _check_served(tabs, _union(batches[i]), samples[i], want, i, ctx)
    srv.close()


def test_hbm_budget_admission(kh, ctx):
    """A budget that holds only a few samples' tables: requests wait for
    memory freed by finalize instead of failing, and every result is exact."""
    samples = _samples(6, seed=31, reads_per_genome=300)
    want = _oracle_tables("budget", samples)
    rng = np.random.default_rng(4)
    budget = 700 << 20  # first tables of a sample: 160 MB
    srv = kh.Server(KS, hbm_budget=budget, max_active=8, chunk_reads=600,
                    batch_bases=200_000)
    batches = {i: _split(r, rng, 2) for i, r in enumerate(samples)}
    tickets = {i: [srv.submit(50 + i, b) for b in bs] for i, bs in batches.items()}
    for i in batches:  # the client finalizes each sample once it is complete
        for t in tickets[i]:
            srv.wait(t)
        print("before finalize", i, srv.stats(), flush=True)
        tabs = srv.finalize(50 + i)
        _check_served(tabs, _union(batches[i]), samples[i], want, i, ctx)
        for t in tabs:
            t.free()
    st = srv.stats()
    print("stats", st, flush=True)
    assert st["completed"] == 12
    assert st["peak_bytes"] <= budget
    srv.close()


def test_heavy_hitters_in_serving(kh):
    pairs = [("A" * 120, "I" * 120)] * 900
    rng = np.random.default_rng(3)
    for _ in range(300):
        s = "".join(rng.choice(list("ACGT"), size=120))
        pairs.append(("AC" * 20 + s[:80], "I" * 120))
    reads = synth.Reads.from_strings(pairs)
    srv = kh.Server((21,), max_active=2, chunk_reads=97, batch_bases=20_000)
    parts = _split(reads, rng, 4)
    ts = [srv.submit(1, p) for p in parts]
    for t in ts:
        srv.wait(t)
    got = srv.finalize(1)[0].to_numpy()
    assert_same_table(got, oracle.count(reads, 21))
    assert got["counts"].max() >= 4096
    srv.close()


def test_server_errors(kh):
    with pytest.raises(kh.KHError) as e:
        kh.Server((21,), use_bloom=True)
    assert e.value.code == kh.KH_EINVAL
    with pytest.raises(kh.KHError):
        kh.Server((22,))
    srv = kh.Server((21,), max_active=1, queue_cap=1)
    with pytest.raises(kh.KHError) as e:
        srv.finalize(12345)
    assert e.value.code == kh.KH_ENOTFOUND
    big = synth.config(2, scale=0.01)
    small = synth.config(1, scale=0.01)
    codes = []
    tickets = [srv.submit(1, big)]
    for _ in range(50):
        try:
            tickets.append(srv.submit(2, small))
        except kh.KHError as ex:
            codes.append(ex.code)
    assert kh.KH_EAGAIN in codes  # the queue holds one request
    for t in tickets:
        srv.wait(t)
    srv.finalize(1)
    if len(tickets) > 1:  # some small batch got in once the queue drained
        srv.finalize(2)
    with pytest.raises(kh.KHError) as e:
        srv.poll(999999)
    assert e.value.code == kh.KH_ENOTFOUND
    srv.close()


def test_empty_batches(kh):
    srv = kh.Server((21, 33))
    empty = synth.Reads(np.zeros(0, np.uint8), np.zeros(0, np.uint8),
                        np.zeros(1, np.int64))
    srv.wait(srv.submit(5, empty))
    tabs = srv.finalize(5)
    assert all(t.info()["n_rows"] == 0 for t in tabs)
    srv.close()
