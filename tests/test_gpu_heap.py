"""Device heap: new/delete (Alg. 1 with request coalescing), quiescent
reclamation, enumeration and do-all, checked against the definitions of the
block states (Sec. 2), brute-force scans of the raw bitmaps, and the oracle's
ideal block counts."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd.heap import Heap  # noqa: E402


def live_set(heap, t=None):
    raw = heap.raw()
    ob = raw["obj_bitmap"].cpu().numpy().view(np.uint64)
    bt = raw["block_type"].cpu().numpy().view(np.uint32)
    out = set()
    for b in np.nonzero(ob)[0]:
        if t is not None and bt[b] != t:
            continue
        w = int(ob[b])
        for s in range(64):
            if (w >> s) & 1:
                out.add(int(b) * 64 + s)
    return out


@pytest.mark.parametrize("cap", [64, 32])
def test_bulk_alloc_dense_and_distinct(cap):
    M = 4096
    heap = Heap(M, cap, [(4, 4, 4)])
    n = 65536 if cap == 64 else 65536 // 2
    h = heap.alloc_n(0, n).cpu().numpy().view(np.uint32)
    assert (h != C.NULL).all()
    assert len(np.unique(h)) == n                           # I1: no slot handed out twice
    assert ((h & 63) < cap).all()
    assert live_set(heap) == set(h.tolist())
    st = heap.stats()
    assert st["live"] == [n] and st["allocs"] == [n] and st["frees"] == [0]
    # Dense policy: every wavefront of 64 lanes fills fresh blocks completely.
    assert st["allocated_blocks"] == [n // cap] and st["active_blocks"] == [0]
    assert heap.check() == {}


def test_ragged_alloc_and_oom():
    # 1,124 requests on a heap of 1,024 slots: out of memory is decided by the
    # free-block count, so a request fails only once every slot is taken --
    # exactly 100 NULL handles, whatever the wavefronts' interleaving.
    heap = Heap(16, 64, [(4,)])
    total = 16 * 64 + 100
    h = heap.alloc_n(0, total).cpu().numpy().view(np.uint32)
    ok = h[h != C.NULL]
    assert len(np.unique(ok)) == len(ok)                    # I1
    assert len(ok) == 16 * 64 and (h == C.NULL).sum() == 100
    st = heap.stats(raise_sticky=False)
    assert st["oom"] == 1 and st["status"] == C.ERR_OOM and st["free_blocks"] == 0
    assert st["retry_limit_hit"] == 0
    assert st["live"] == [16 * 64]
    assert st["blocks_taken"] == 16 and st["blocks_returned"] == 0
    assert heap.alloc_n(0, 1).cpu().numpy().view(np.uint32)[0] == C.NULL
    chk = heap.check()
    assert chk == {"sticky": "DSOAR_ERR_OOM"}


def test_free_count_keeps_a_request_looking_when_the_summary_lags():
    # The state an online release passes through: a block's free bit is set
    # at level 0 but not yet in the word above it.  Made here from the host
    # on a full heap (one block emptied and reclaimed, so the free-block count
    # is 1, then its top-level bit cleared): the free bitmap's top word reads
    # 0 while one block is free.  A request must not report out of memory:
    # it either gets that block or gives up with the retry-limit flag, and
    # its kernel ends.
    M = 4096
    heap = Heap(M, 64, [(4,)])
    h = heap.alloc_n(0, M * 64).cpu().numpy().view(np.uint32)
    assert (h != C.NULL).all()
    victim = 1234
    heap.free_n(torch.from_numpy(h[(h >> 6) == victim].view(np.int32)).cuda())
    heap.reclaim()
    st = heap.stats()
    assert st["free_blocks"] == 1 and M + st["blocks_returned"] - st["blocks_taken"] == 1
    L = heap.layout()
    assert L.num_levels == 2
    words = heap.raw()["bitmaps"][0]          # the free bitmap, all levels
    top = L.level_word_offset[1]
    assert int(words[top].item()) == 1 << (victim // 64) and int(words[victim // 64].item()) == 1 << (victim % 64)
    words[top] = 0                            # the summary now lags level 0
    torch.cuda.synchronize()
    got = heap.alloc_n(0, 64).cpu().numpy().view(np.uint32)
    st = heap.stats(raise_sticky=False)
    assert st["oom"] == 0
    handed = got[got != C.NULL]
    assert ((handed >> 6) == victim).all()
    assert len(handed) == 64 or st["retry_limit_hit"] == 1


def test_fragmentation_against_the_ideal_heap_model():
    # Allocated blocks after random churn, against the oracle heap model's
    # ideal (the dense policy of Sec. 2.2 run sequentially: lowest active
    # block, lowest slot) for the same live count: never fewer than
    # ceil(live / 64), and reported, not compared, beyond that.
    import oracle
    rng = np.random.default_rng(5)
    M = 1024
    heap = Heap(M, 64, [(4,)])
    h = heap.alloc_n(0, 40000).cpu().numpy().view(np.uint32)
    kill = h[rng.random(h.size) < 0.5]
    heap.free_n(torch.from_numpy(kill.view(np.int32)).cuda())
    again = heap.alloc_n(0, 10000).cpu().numpy().view(np.uint32)
    assert (again != C.NULL).all()
    st = heap.stats()
    live = st["live"][0]
    assert live == 40000 - kill.size + 10000
    model = oracle.HeapModel(M, 64, 1)
    handles = [model.alloc(0) for _ in range(40000)]
    for i in np.nonzero(np.isin(h, kill))[0]:
        assert model.free(handles[i])
    for _ in range(10000):
        model.alloc(0)
    model.reclaim()
    ideal = model.counts()[0]["allocated_blocks"]
    assert model.counts()[0]["live"] == live
    gpu = st["allocated_blocks"][0]
    assert gpu >= -(-live // 64) and ideal >= -(-live // 64)
    print(f"fragmentation: {gpu} allocated blocks on the device, {ideal} in the sequential model, "
          f"{-(-live // 64)} at full density, for {live} objects")
    assert heap.check() == {}


@pytest.mark.parametrize("policy,blocks", [(C.POLICY_DENSE, 1), (C.POLICY_FRESH, 2)])
def test_type_policy_fresh_opens_own_blocks(policy, blocks):
    # Two requests of 10: the dense policy puts the second into the block the
    # first left active; the fresh policy opens a block for each.
    heap = Heap(64, 64, [(4,)])
    heap.set_type_policy(0, policy)
    a = heap.alloc_n(0, 10).cpu().numpy().view(np.uint32)
    b = heap.alloc_n(0, 10).cpu().numpy().view(np.uint32)
    h = np.concatenate([a, b])
    assert (h != C.NULL).all() and len(np.unique(h)) == 20
    st = heap.stats()
    assert st["live"] == [20] and st["allocated_blocks"] == [blocks] and st["active_blocks"] == [blocks]
    assert heap.check() == {}


@pytest.mark.parametrize("policy,active_after", [(C.POLICY_DENSE, 1), (C.POLICY_BOUNDED, 17)])
def test_type_policy_bounded_stops_after_two_lookups(policy, active_after):
    # 32 full blocks with one hole each (all under one level-0 word), then one
    # wavefront asks for 64: each lookup reserves in up to 8 of those blocks.
    # Dense fills all 32 holes (four lookups) and opens one block for the other
    # 32; bounded stops after two lookups (16 holes) and opens one block for 48.
    heap = Heap(64, 64, [(4,)])
    heap.set_type_policy(0, policy)
    h = heap.alloc_n(0, 32 * 64)
    hn = np.sort(h.cpu().numpy().view(np.uint32))
    holes = hn[np.arange(32 * 64) % 64 == 5]
    heap.free_n(torch.from_numpy(holes.view(np.int32)).to(h.device))
    assert heap.stats()["active_blocks"] == [32]
    got = heap.alloc_n(0, 64).cpu().numpy().view(np.uint32)
    assert (got != C.NULL).all() and len(np.unique(got)) == 64
    st = heap.stats()
    assert st["live"] == [32 * 64 + 32] and st["allocated_blocks"] == [33]
    assert st["active_blocks"] == [active_after]
    assert len(set(got.tolist()) & set(holes.tolist())) == 64 - (32 if policy == C.POLICY_DENSE else 48)
    assert heap.check() == {}


@pytest.mark.parametrize("policy", [C.POLICY_FRESH, C.POLICY_BOUNDED])
def test_type_policy_falls_back_to_active_blocks(policy):
    # Every block full, then 10 slots freed in each: no free block is left,
    # so fresh and bounded requests must take the freed slots, all of them,
    # before OOM.
    heap = Heap(16, 64, [(4,)])
    heap.set_type_policy(0, policy)
    h = heap.alloc_n(0, 16 * 64)
    hn = h.cpu().numpy().view(np.uint32)
    assert (hn != C.NULL).all()
    freed = torch.from_numpy(np.sort(hn)[np.arange(16 * 64) % 64 < 10].view(np.int32)).to(h.device)
    heap.free_n(freed)
    st = heap.stats()
    assert st["live"] == [16 * 64 - 160] and st["free_blocks"] == 0 and st["active_blocks"] == [16]
    again = heap.alloc_n(0, 160).cpu().numpy().view(np.uint32)
    assert (again != C.NULL).all()
    assert set(again.tolist()) == set(freed.cpu().numpy().view(np.uint32).tolist())
    st = heap.stats(raise_sticky=False)
    assert st["live"] == [16 * 64] and st["oom"] == 0
    assert heap.alloc_n(0, 1).cpu().numpy().view(np.uint32)[0] == C.NULL
    assert heap.check() == {"sticky": "DSOAR_ERR_OOM"}


@pytest.mark.parametrize("cap,ntypes", [(64, 1), (64, 3), (32, 2)])
def test_churn_invariants_and_visits(cap, ntypes):
    rng = np.random.default_rng(cap + ntypes)
    M = 512
    heap = Heap(M, cap, [(4, 8)] * ntypes)
    live = {}
    for rnd in range(6):
        for t in range(ntypes):
            n = int(rng.integers(1, 3000))
            h = heap.alloc_n(t, n).cpu().numpy().view(np.uint32)
            h = h[h != C.NULL]
            for x in h.tolist():
                assert x not in live
                live[x] = t
        # delete a random subset (grouped by block inside the kernel)
        keys = np.array(sorted(live), dtype=np.uint32)
        kill = keys[rng.random(len(keys)) < 0.5]
        heap.free_n(torch.tensor(kill.view(np.int32), device="cuda"))
        for x in kill.tolist():
            del live[x]
        st = heap.stats()
        for t in range(ntypes):
            assert st["live"][t] == sum(1 for v in live.values() if v == t)
            assert st["live"][t] == st["allocs"][t] - st["frees"][t]
        assert live_set(heap) == set(live)
        for t in range(ntypes):
            # I8: the do-all visits each live object once and nothing else.
            counts = heap.visit_counts(t).cpu().numpy()
            exp = np.zeros(M * 64, dtype=np.int32)
            idx = [x for x, v in live.items() if v == t]
            exp[idx] = 1
            assert np.array_equal(counts, exp)
        assert heap.check() == {}
        st = heap.stats()
        for t in range(ntypes):
            assert st["allocated_blocks"][t] >= -(-st["live"][t] // cap)


def test_double_free_flagged():
    heap = Heap(8, 64, [(4,)])
    h = heap.alloc_n(0, 10)
    heap.free_n(h[:3])
    heap.free_n(h[:1])
    st = heap.stats(raise_sticky=False)
    assert st["double_free"] == 1 and st["live"] == [7] and st["frees"] == [3]


def test_field_roundtrip_and_delete_if_mod():
    heap = Heap(64, 64, [(4, 4)])
    h = heap.alloc_n(0, 1000)
    ids = torch.arange(1000, dtype=torch.int32, device="cuda")
    heap.field_write(0, 0, h, ids)
    heap.field_write(0, 1, h, ids * 7)
    assert torch.equal(heap.field_read(0, 1, h), ids * 7)
    heap.delete_if_mod(0, 0, 3, 0)
    out, present = heap.gather(0, 0, 1, 1000)
    p = present.cpu().numpy().astype(bool)
    assert np.array_equal(p, np.arange(1000) % 3 != 0)
    assert np.array_equal(out.cpu().numpy()[p], (np.arange(1000) * 7)[p])
    assert heap.check() == {}


def test_field_access_skips_handles_outside_the_heap():
    # 8 blocks of 32 slots: a slot >= 32, a block >= 8, NULL and a block near
    # the top of the handle range are skipped by reads and writes alike.
    heap = Heap(8, 32, [(4,)])
    h = heap.alloc_n(0, 3)
    heap.field_write(0, 0, h, torch.tensor([7, 8, 9], dtype=torch.int32, device="cuda"))
    bad = torch.tensor([40, 8 << 6, -1, ((1 << 26) - 2) << 6], dtype=torch.int64).to(torch.int32).cuda()
    heap.field_write(0, 0, bad, torch.full((4,), 5, dtype=torch.int32, device="cuda"))
    objs = torch.cat([h, bad])
    assert heap.field_read(0, 0, objs).cpu().tolist() == [7, 8, 9, 0, 0, 0, 0]
    assert heap.stats()["live"] == [3]
    assert heap.check() == {}


def test_enumeration_matches_brute_force_and_reclaims():
    rng = np.random.default_rng(3)
    M = 3000  # ragged: not a multiple of 64, several scan tiles
    heap = Heap(M, 64, [(4,), (4,)])
    a = heap.alloc_n(0, 100000)
    b = heap.alloc_n(1, 50000)
    kill = a[torch.tensor(rng.random(100000) < 0.7, device="cuda")]
    heap.free_n(kill)
    heap.free_n(b)                                           # type 1 becomes empty
    heap.enumerate(0)
    cnt = heap.enum_count(0)
    R, S = heap.enum_arrays(0, cnt)
    raw = heap.raw()
    ob = raw["obj_bitmap"].cpu().numpy().view(np.uint64)
    bt = raw["block_type"].cpu().numpy()
    exp_blocks = [i for i in range(M) if bt[i] == 0 and ob[i] != 0]
    assert R.cpu().numpy().tolist() == exp_blocks            # ascending, exactly the non-empty blocks
    assert np.array_equal(S.cpu().numpy().view(np.uint64), ob[exp_blocks])
    heap.enumerate(1)
    assert heap.enum_count(1) == 0
    st = heap.stats()
    assert st["allocated_blocks"][1] == 0 and st["typed_blocks"][1] == 0
    assert heap.check() == {}
    # reused blocks take the other type after reclamation
    c = heap.alloc_n(1, 64 * 10)
    assert (c.cpu().numpy().view(np.uint32) != C.NULL).all()
    assert heap.check() == {}


@pytest.mark.parametrize("flags", [C.DO_PERSISTENT, C.DO_PLAIN])
def test_enumeration_large_many_tiles(flags):
    M = 1 << 18  # 4096 level-0 words, 128 scan tiles, 3 levels
    heap = Heap(M, 64, [(4,)])
    n = 3_000_000
    h = heap.alloc_n(0, n)
    keep = torch.rand(n, device="cuda") < 0.5
    heap.free_n(h[~keep])
    counts = heap.visit_counts(0, flags)
    exp = torch.zeros(M * 64, dtype=torch.int32, device="cuda")
    exp[h[keep].long()] = 1
    assert torch.equal(counts, exp)
    assert heap.check() == {}
