"""kh_count_noalloc, the entry point that allocates no device memory (every
buffer is carved from the library's fixed per-device scratch array), against
kh_count + kh_table_export on the same reads: bit-identical rows on two
calls in a row, the second with a smaller input (the scratch keeps the first
call's contents, so anything that must start at zero has to be cleared),
with and without the Bloom screen, at one- to four-word keys; and the
documented errors."""
import numpy as np
import pytest

import synth
from brute import assert_same_table

pytestmark = pytest.mark.gpu


def _outs(n, k):
    import torch
    W = (k + 31) // 32
    return (torch.zeros((n, W), dtype=torch.int64, device="cuda"),
            torch.zeros(n, dtype=torch.int32, device="cuda"),
            torch.zeros((n, 8), dtype=torch.int32, device="cuda"),
            torch.zeros((n, 2), dtype=torch.uint8, device="cuda"))


def _rows(outs, n, k):
    keys, counts, ext, codes = outs
    return dict(k=k, W=(k + 31) // 32, n_rows=n,
                keys=keys[:n].cpu().numpy().view(np.uint64),
                counts=counts[:n].cpu().numpy().view(np.uint32),
                ext=ext[:n].cpu().numpy().view(np.uint32),
                codes=codes[:n].cpu().numpy())


@pytest.fixture(scope="module")
def ctx(kh):
    c = kh.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("k,bloom", [(21, False), (21, True), (33, True), (55, False),
                                     (77, False), (99, True)])
def test_noalloc_equals_count(kh, ctx, k, bloom):
    big = kh.DeviceReads.from_host(synth.config(1))              # 6,667 reads
    small = kh.DeviceReads.from_host(synth.config(1, scale=0.2))  # 1,333 reads
    for reads in (big, small):  # the second call reuses the dirty scratch
        want = ctx.count(reads, k, use_bloom=bloom).to_numpy()
        outs = _outs(want["n_rows"] + 17, k)
        n, nw = kh.count_noalloc(reads, k, *outs, use_bloom=bloom)
        print("k=%d bloom=%d rows=%d windows=%d" % (k, bloom, n, nw), flush=True)
        assert n == want["n_rows"] and nw == want["n_windows"]
        assert_same_table(_rows(outs, n, k), want)
        assert not outs[1][n:].any()  # nothing written past the rows


def test_noalloc_output_too_small(kh, ctx):
    reads = kh.DeviceReads.from_host(synth.config(1, scale=0.3))
    want = ctx.count(reads, 21).to_numpy()
    small = _outs(want["n_rows"] - 1, 21)
    with pytest.raises(kh.KHError) as e:
        kh.count_noalloc(reads, 21, *small)
    assert e.value.code == kh.KH_EOVERFLOW and e.value.needed == want["n_rows"]
    outs = _outs(want["n_rows"], 21)
    n, _ = kh.count_noalloc(reads, 21, *outs)
    assert_same_table(_rows(outs, n, 21), want)


def test_noalloc_limits(kh):
    import torch
    outs = _outs(16, 21)
    # more bases than the documented limit: refused before any launch
    n = kh.NOALLOC_MAX_BASES + 1
    seq = torch.full((n,), ord("A"), dtype=torch.uint8, device="cuda")
    off = torch.tensor([0, n], dtype=torch.int64, device="cuda")
    with pytest.raises(kh.KHError) as e:
        kh.count_noalloc(kh.DeviceReads(seq, seq, off), 21, *outs)
    assert e.value.code == kh.KH_EINVAL
    del seq
    # more distinct k-mers than the scratch's table holds
    rng = np.random.default_rng(5)
    g = rng.choice(np.frombuffer(b"ACGT", np.uint8), size=6_000_000)
    reads = synth.Reads(g, np.full(g.shape, ord("I"), np.uint8),
                        np.arange(0, g.size + 1, 150, dtype=np.int64))
    with pytest.raises(kh.KHError) as e:
        kh.count_noalloc(kh.DeviceReads.from_host(reads), 21, *outs, min_count=1)
    assert e.value.code == kh.KH_ENOMEM
    # host reads are refused; empty reads give no rows
    with pytest.raises(ValueError):
        kh.count_noalloc(synth.config(1, scale=0.01), 21, *outs)
    empty = kh.DeviceReads.from_host(synth.Reads(np.zeros(0, np.uint8), np.zeros(0, np.uint8),
                                                 np.zeros(1, np.int64)))
    assert kh.count_noalloc(empty, 21, *outs) == (0, 0)
    # and the entry point still counts correctly after the failures
    r = kh.DeviceReads.from_host(synth.config(1, scale=0.1))
    out2 = _outs(20000, 33)
    n2, _ = kh.count_noalloc(r, 33, *out2)
    assert n2 > 0
