"""The owner-partitioned count (kh_tuning partitioned = 1) where it differs
from the single-table path: owners whose keys do not fit their LDS table are
split finer and counted again, and when even the finest split does not fit
the k is counted on the single-table path.  Both are forced from the host
with the KMERHIP_OWNER_SLOTS hook (fewer LDS slots per owner than owners
are sized for); every table must equal the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from brute import assert_same_table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def octx(kh):
    c = kh.Context(0)
    assert c.tuning()["partitioned"] == 1
    yield c
    c.close()


def _random_reads(seed, n, length):
    rng = np.random.default_rng(seed)
    pairs = []
    for _ in range(n):
        s = "".join(rng.choice(list("ACGT"), size=length))
        pairs.append((s, "I" * length))
    return synth.Reads.from_strings(pairs)


def test_resplit_when_owners_overflow(octx, monkeypatch):
    """Coverage ~1, no Bloom screen, 900,000 windows: owners are sized for
    the full LDS table (1,344 records at k = 21, so ~880 per level-1 bucket
    and no level-2 split) but get 700 slots, so they overflow and are split
    by more key bits, which fits.  With min_count = 1 every key is a row, so
    the rows are staged in a buffer of their own."""
    reads = _random_reads(3, 9000, 120)
    want = oracle.count(reads, 21, min_count=1)
    monkeypatch.setenv("KMERHIP_OWNER_SLOTS", "700")
    got = octx.count(reads, 21, min_count=1).to_numpy()
    st = octx.stats()
    assert st["rebuilds"] >= 1 and st["heavy"] > 0
    assert st["table_bytes"] > 2 * 8 * got["n_windows"]
    assert_same_table(got, want)
    assert got["n_windows"] == want["n_windows"]


def test_staging_runs_out(octx):
    """Every read twice, min_count = 2, no Bloom screen: half the windows
    are rows, more than the level-1 record buffer stages (8 bytes per
    record, 46 per row at k = 21), so the owner pass runs again with every
    owner's rows at its scanned offset."""
    reads = _random_reads(5, 4000, 120)
    reads = synth.Reads.from_strings(reads.strings() * 2)
    want = oracle.count(reads, 21, min_count=2)
    got = octx.count(reads, 21, min_count=2).to_numpy()
    st = octx.stats()
    assert st["table_bytes"] > 2 * 8 * got["n_windows"]  # the second staging
    assert st["rebuilds"] == 0
    assert_same_table(got, want)
    assert got["n_windows"] == want["n_windows"]


def test_unfit_owner_falls_back(octx, monkeypatch):
    """200 distinct 21-mers sharing their top 12 bases (all in one owner at
    any split depth), each read twice: with 16 slots per owner they never
    fit and the k is counted on the single-table path; with the full LDS
    table they fit.  The same rows either way."""
    rng = np.random.default_rng(9)
    pairs = []
    for _ in range(200):
        s = "A" * 12 + "".join(rng.choice(list("ACG"), size=9))
        pairs += [(s, "I" * 21)] * 2
    pairs += _random_reads(4, 300, 100).strings()
    reads = synth.Reads.from_strings(pairs)
    want = oracle.count(reads, 21)
    got = octx.count(reads, 21, use_bloom=True).to_numpy()
    assert_same_table(got, want)
    monkeypatch.setenv("KMERHIP_OWNER_SLOTS", "16")
    got = octx.count(reads, 21, use_bloom=True).to_numpy()
    assert_same_table(got, want)
    tabs = octx.count_multi_k(reads, [21, 33], use_bloom=True)
    assert_same_table(tabs[0].to_numpy(), want)
    assert_same_table(tabs[1].to_numpy(), oracle.count(reads, 33))


@pytest.mark.parametrize("k", [21, 55, 99])
def test_key_space_part(octx, k):
    """A key-space part (owner_shards): only the part's windows are routed."""
    reads = synth.config(1, scale=0.3)
    got = octx.count(reads, k, use_bloom=True, owner_shards=3, owner=1).to_numpy()
    want = oracle.count_shard(reads, k, 3, 1)
    assert_same_table(got, want, totals=False)
    assert got["n_windows"] == want["n_windows"]


def test_metagenome_sample_both_paths(kh, octx):
    """A 100,000-read sample of the benchmark's metagenome at every k of the
    benchmark: the owner path equals the single-table path (each is checked
    against the oracle elsewhere), and the oracle at k = 21."""
    reads = synth.config(2, scale=0.01)
    ks = [21, 33, 55, 77, 99]
    single = kh.Context(0)
    single.set_tuning(partitioned=0)
    try:
        want = {k: single.count(reads, k, use_bloom=True).to_numpy() for k in ks}
    finally:
        single.close()
    dev = kh.DeviceReads.from_host(reads)
    for k, t in zip(ks, octx.count_multi_k(dev, ks, use_bloom=True)):
        got = t.to_numpy()
        assert_same_table(got, want[k])
        assert got["n_windows"] == want[k]["n_windows"]
        t.free()
    assert_same_table(want[21], oracle.count(reads, 21))
