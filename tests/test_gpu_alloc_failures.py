"""A refused device allocation at every point of a batched call (through the
caller-allocator hooks): the call either reports KH_ENOMEM or, when the
refusal hits the batched path, counts the k one after another (finishing a
streamed upload first) and returns the oracle's tables.  Every block the
context drew is handed back when it is destroyed."""
import pytest

import oracle
import synth
from brute import assert_same_table

pytestmark = pytest.mark.gpu

KS = [21, 33, 77]


def _allocator(refuse):
    import torch
    st = {"n": 0, "refused": 0, "live": {}}

    def alloc(nbytes, device):
        st["n"] += 1
        if st["n"] in refuse:  # the pool retries once after dropping its cache
            st["refused"] += 1
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes, device)
        st["live"][p] = nbytes
        return p

    def free(ptr, nbytes, device):
        assert st["live"].pop(ptr) == nbytes
        torch.cuda.caching_allocator_delete(ptr)

    return (alloc, free), st


@pytest.mark.parametrize("partitioned", [0, 1])
def test_refusal_at_every_allocation(kh, monkeypatch, partitioned):
    """Single-table path: a refusal in the batched call falls back to the k
    one after another, so some refusals still give the oracle's tables.
    Owner path: a refusal of one of its own buffers counts that k on the
    single-table path.  Every refusal gives KH_ENOMEM or the oracle's
    tables."""
    monkeypatch.setenv("KMERHIP_STREAM_CHUNK", "8192")
    reads = synth.config(1, scale=0.3)
    want = {k: oracle.count(reads, k) for k in KS}
    hooks, st = _allocator(set())
    ctx = kh.Context(0, allocator=hooks)
    ctx.set_tuning(partitioned=partitioned)
    ctx.count_multi_k(reads, KS, use_bloom=True)  # dry run: how many allocations
    total = st["n"]
    ctx.close()
    assert not st["live"]
    outcomes = {"ok": 0, "enomem": 0}
    for n in range(3, total + 1):  # 1, 2: the context's own counters
        hooks, st = _allocator({n, n + 1})
        ctx = kh.Context(0, allocator=hooks)
        ctx.set_tuning(partitioned=partitioned)
        try:
            tabs = ctx.count_multi_k(reads, KS, use_bloom=True)
        except kh.KHError as e:
            assert e.code == kh.KH_ENOMEM, str(e)
            outcomes["enomem"] += 1
        else:
            for k, t in zip(KS, tabs):
                assert_same_table(t.to_numpy(), want[k])
                t.free()
            outcomes["ok"] += 1
        ctx.close()
        assert not st["live"], "blocks not handed back (refusal at %d)" % n
    print("allocations per call:", total, "outcomes:", outcomes, flush=True)
    assert outcomes["ok"] > 0
