"""Device memory from the caller's allocator (kh_create's alloc_fn/free_fn):
tables bit-identical to the oracle's, every block drawn through the hooks
and handed back by the time the context is destroyed, and a refusing
allocator reported as KH_ENOMEM without harm to the context."""
import pytest

import oracle
import synth
from brute import assert_same_table

pytestmark = pytest.mark.gpu


def test_torch_caching_allocator(kh):
    import torch
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    reads = synth.config(1)
    ctx = kh.Context(0, allocator="torch")
    try:
        for k in (21, 55):
            t = ctx.count(reads, k, use_bloom=True)
            assert_same_table(t.to_numpy(), oracle.count(reads, k))
            t.free()
        assert torch.cuda.memory_allocated(0) > base  # the pool's blocks are torch's
    finally:
        ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == base


def test_hooks_see_every_block(kh):
    import torch
    live = {}
    log = {"alloc": 0, "free": 0}

    def alloc(nbytes, device):
        assert device == 0
        p = torch.cuda.caching_allocator_alloc(nbytes, device)
        live[p] = nbytes
        log["alloc"] += 1
        return p

    def free(ptr, nbytes, device):
        assert live.pop(ptr) == nbytes
        log["free"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    reads = synth.config(2, scale=0.01)
    ks = [21, 33, 77]
    ctx = kh.Context(0, allocator=(alloc, free))
    try:
        tabs = ctx.count_multi_k(kh.DeviceReads.from_host(reads), ks, use_bloom=True)
        for k, t in zip(ks, tabs):
            assert_same_table(t.to_numpy(), oracle.count(reads, k))
            t.free()
        assert log["alloc"] > 0 and live
        ctx.trim()  # free blocks go back at once
        n_after_trim = len(live)
        assert log["free"] > 0 and n_after_trim < log["alloc"]
    finally:
        ctx.close()
    assert not live and log["free"] == log["alloc"]


def test_refusing_allocator(kh):
    import torch
    budget = {"left": 1 << 20}  # far too little for any count
    live = {}

    def alloc(nbytes, device):
        if nbytes > budget["left"]:
            return 0
        budget["left"] -= nbytes
        p = torch.cuda.caching_allocator_alloc(nbytes, device)
        live[p] = nbytes
        return p

    def free(ptr, nbytes, device):
        budget["left"] += live.pop(ptr)
        torch.cuda.caching_allocator_delete(ptr)

    reads = synth.config(1, scale=0.2)
    ctx = kh.Context(0, allocator=(alloc, free))
    try:
        with pytest.raises(kh.KHError) as e:
            ctx.count(reads, 21, use_bloom=True)
        assert e.value.code == kh.KH_ENOMEM
        budget["left"] += 1 << 30  # the framework made room
        t = ctx.count(reads, 21, use_bloom=True)
        assert_same_table(t.to_numpy(), oracle.count(reads, 21))
        t.free()
    finally:
        ctx.close()
    assert not live
