"""Key-space parts (the one-GPU share of a multi-GPU run): counting only
the k-mers a part owns gives exactly the oracle's shard, and the parts
together give the whole table."""
import numpy as np
import pytest

import oracle
import synth
from brute import assert_same_table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def w1():
    return synth.config(1, scale=0.3)


@pytest.fixture(scope="module")
def sctx(kh):
    c = kh.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("k", [21, 33, 77, 99])
@pytest.mark.parametrize("bloom", [False, True])
def test_parts_equal_oracle_shards(kh, sctx, w1, k, bloom):
    S = 5
    full = oracle.count(w1, k)
    total = 0
    rows = 0
    for s in range(S):
        got = sctx.count(w1, k, use_bloom=bloom, owner_shards=S, owner=s).to_numpy()
        want = oracle.count_shard(w1, k, S, s)
        assert_same_table(got, want, totals=False)
        assert got["n_windows"] == want["n_windows"]
        for i in range(0, got["n_rows"], max(1, got["n_rows"] // 20)):
            assert kh.owner_of(got["keys"][i], S) == s
        total += got["n_windows"]
        rows += got["n_rows"]
    assert total == full["n_windows"] and rows == full["n_rows"]


def test_parts_in_the_batched_call(kh, sctx, w1):
    ks = [21, 55, 99]
    S, s = 8, 3
    tabs = sctx.count_multi_k(w1, ks, use_bloom=True, owner_shards=S, owner=s)
    for k, t in zip(ks, tabs):
        assert_same_table(t.to_numpy(), oracle.count_shard(w1, k, S, s), totals=False)


def test_part_errors(kh, sctx, w1):
    with pytest.raises(kh.KHError) as e:
        sctx.count(w1, 21, owner_shards=4, owner=4)
    assert e.value.code == kh.KH_EINVAL
    with pytest.raises(kh.KHError) as e:
        kh.Server((21,), owner_shards=2, owner=0)
    assert e.value.code == kh.KH_EINVAL
    # one part of one is the whole table
    got = sctx.count(w1, 21, owner_shards=1, owner=0).to_numpy()
    assert_same_table(got, oracle.count(w1, 21))
