"""Large single-GPU share: 200M paired 150 bp reads of a 1,000-genome
metagenome (1-6 Mbp genomes, log-normal(0, 2) abundances, 1 % errors)
counted at k = 33 and 77 with the Bloom screen, as part 0 of 8 of the k-mer
space: the table one GPU of an 8-GPU node would own.  The whole read set is
scanned; only owned k-mers reach the Bloom filter and the table.

Opt-in (KMERHIP_LARGE=1): the reads take about a minute and 65 GB of host
memory to generate, and the oracle rescans all of them for the sampled
checks.  Properties are checked on every row; sampled rows and sampled
windows are recounted exactly by the oracle.
"""
import json
import os
import time

import numpy as np
import pytest

import oracle
import synth
from brute import key_words, revcomp, side_letter
from test_oracle_pins import shard_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("KMERHIP_LARGE") != "1",
                                 reason="opt-in: set KMERHIP_LARGE=1")]

KS = (33, 77)
S, OWNER = 8, 0


@pytest.fixture(scope="module")
def large():
    import torch
    import paper_1809_07014_amd as kh
    t0 = time.time()
    reads = synth.config(5)
    print("generated %d reads in %.1f s" % (reads.n_reads, time.time() - t0), flush=True)
    ctx = kh.Context(0)
    dev = kh.DeviceReads.from_host(reads)
    opts = dict(use_bloom=True, owner_shards=S, owner=OWNER)
    for t in ctx.count_multi_k(dev, KS, **opts):  # warm-up call
        t.free()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tabs = ctx.count_multi_k(dev, KS, **opts)
    torch.cuda.synchronize()
    call_s = time.perf_counter() - t1
    report = dict(call_s=round(call_s, 3), phases_ms=ctx.timing(), per_k={})
    total_windows = sum(reads.n_reads * (151 - k) for k in KS)
    for i, k in enumerate(KS):
        ms, st = ctx.k_report(i)
        report["per_k"][k] = dict(ms=ms, stats=st)
    report["windows_scanned_per_s"] = total_windows / call_s
    print("LARGE", json.dumps(report), flush=True)
    out = {k: t.to_numpy() for k, t in zip(KS, tabs)}
    for t in tabs:
        t.free()
    ctx.close()
    del dev
    return reads, out


@pytest.mark.parametrize("k", KS)
def test_large_properties(large, k):
    reads, tabs = large
    t = tabs[k]
    total = reads.n_reads * (151 - k)
    print("k=%d rows=%d owned windows=%d of %d" % (k, t["n_rows"], t["n_windows"], total),
          flush=True)
    assert abs(t["n_windows"] * S / total - 1.0) < 0.05
    keys = t["keys"]
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
    assert np.all(shard_np(keys, S) == OWNER)
    rng = np.random.default_rng(k)
    for i in rng.choice(t["n_rows"], 2000, replace=False):
        c, e = int(t["counts"][i]), t["ext"][i].tolist()
        assert t["codes"][i].tobytes().decode() == side_letter(e[:4], c) + side_letter(e[4:], c)


def _find(keys, q):
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
def test_large_sampled_exact(large, k):
    reads, tabs = large
    t = tabs[k]
    rng = np.random.default_rng(500 + k)
    rows = rng.choice(t["n_rows"], 12, replace=False)
    q = [t["keys"][r] for r in rows]
    wins = []
    while len(wins) < 12:  # windows whose key this part owns
        r = int(rng.integers(0, reads.n_reads))
        a = int(reads.offsets[r])
        i = int(rng.integers(0, 151 - k))
        w = reads.seq[a + i:a + i + k].tobytes().decode()
        kw = np.array(key_words(min(w, revcomp(w))), np.uint64)
        if int(shard_np(kw.reshape(1, -1), S)[0]) == OWNER:
            wins.append(kw)
    qa = np.concatenate([np.array(q, np.uint64), np.array(wins, np.uint64)])
    # the oracle rescans every read; counts and tallies add over read ranges
    counts = np.zeros(len(qa), np.uint64)
    ext = np.zeros((len(qa), 8), np.uint64)
    step = 20_000_000
    for a in range(0, reads.n_reads, step):
        c, e = oracle.count_keys(reads.slice(a, min(reads.n_reads, a + step)), k, qa)
        counts += c
        ext += e
        print("k=%d oracle scanned %d reads" % (k, min(reads.n_reads, a + step)), flush=True)
    for j, r in enumerate(rows):
        assert int(counts[j]) == int(t["counts"][r])
        assert ext[j].tolist() == t["ext"][r].tolist()
    for j in range(len(wins)):
        c = int(counts[len(rows) + j])
        assert c >= 1
        idx = _find(t["keys"], qa[len(rows) + j])
        if c >= 2:
            assert idx >= 0 and int(t["counts"][idx]) == c
            assert t["ext"][idx].tolist() == ext[len(rows) + j].tolist()
        else:
            assert idx < 0
