"""Pins of the oracle's sequential heap model (paper Sec. 2 block states,
Sec. 2.2 Alg. 1, dense allocation policy)."""
import random

import pytest


def test_dense_policy_fills_blocks_in_order(orc):
    h = orc.HeapModel(16, 64, 1)
    handles = [h.alloc(0) for _ in range(200)]
    # Alg. 1 with lowest-first choices: objects fill block 0, then 1, ...
    assert handles == list(range(200))
    c = h.counts()[0]
    assert c["allocated_blocks"] == 4            # ceil(200 / 64): fully dense
    assert c["active_blocks"] == 1               # only the partial block is active
    assert h.check() == []


def test_alloc_prefers_active_block(orc):
    h = orc.HeapModel(8, 64, 1)
    hs = [h.alloc(0) for _ in range(128)]        # blocks 0 and 1 full
    assert h.counts()[0]["active_blocks"] == 0
    assert h.free(hs[70])                        # block 1 not full any more
    assert h.counts()[0]["active_blocks"] == 1
    assert h.alloc(0) == 70                      # reuses the active block's hole
    assert h.counts()[0]["active_blocks"] == 0


def test_types_do_not_share_blocks(orc):
    h = orc.HeapModel(8, 64, 2)
    a = h.alloc(0)
    b = h.alloc(1)
    assert a // 64 != b // 64
    assert h.check() == []


def test_oom_exactly_at_capacity(orc):
    h = orc.HeapModel(4, 32, 1)
    hs = [h.alloc(0) for _ in range(4 * 32)]
    assert len(set(hs)) == 128 and min(hs) >= 0
    assert h.alloc(0) == -1                      # out of memory
    assert all(hh % 64 < 32 for hh in hs)        # slots stay below the capacity


def test_reclaim_returns_empty_blocks(orc):
    h = orc.HeapModel(8, 64, 2)
    hs = [h.alloc(0) for _ in range(130)]
    for x in hs:
        h.free(x)
    assert h.check() != []                       # empty blocks still allocated
    assert h.reclaim() == 3
    assert h.check() == []
    assert h.counts()["free_blocks"] == 8
    assert h.alloc(1) == 0                       # a reclaimed block takes a new type


def test_double_free_rejected(orc):
    h = orc.HeapModel(2, 64, 1)
    x = h.alloc(0)
    assert h.free(x)
    assert not h.free(x)


@pytest.mark.parametrize("cap", [32, 64])
def test_random_churn_invariants(orc, cap):
    rnd = random.Random(cap)
    M = 64
    h = orc.HeapModel(M, cap, 3)
    live = {}
    for it in range(6000):
        if live and rnd.random() < 0.45:
            x = rnd.choice(list(live))
            assert h.free(x)
            del live[x]
        else:
            t = rnd.randrange(3)
            x = h.alloc(t)
            if x == -1:
                continue
            assert x not in live                 # I1: no slot handed out twice
            live[x] = t
        if it % 500 == 0:
            h.reclaim()
            assert h.check() == []               # I2..I7 at quiescence
    h.reclaim()
    assert h.check() == []
    c = h.counts()
    for t in range(3):
        assert c[t]["live"] == sum(1 for v in live.values() if v == t)
        assert c[t]["live"] == c[t]["allocs"] - c[t]["frees"]
    ob, bt = h.dump()
    # Brute force: the set of live handles equals the set bits of the bitmaps.
    bits = {b * 64 + s for b in range(M) for s in range(64) if (int(ob[b]) >> s) & 1}
    assert bits == set(live)
    for x, t in live.items():
        assert bt[x // 64] == t
