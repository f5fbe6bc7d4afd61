"""Online block reclamation: the delete that empties a block frees it inside
the kernel, so blocks change type under concurrent allocation.  A stress
kernel interleaves new and delete of four types; every slot must be handed
out once (kept handles distinct, each object's field 0 still holding its own
handle, live counts exact) and every invariant must hold afterwards.  With
online reclamation a heap half the size that the per-type blocks would need
completes; without it the same run runs out of blocks.  The applications give
the oracle's results with online reclamation on."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd import apps  # noqa: E402
from paper_1809_07444_amd.heap import Heap  # noqa: E402
from synth import workloads as W  # noqa: E402

TYPES = [(4,), (4, 4), (4, 4, 4), (4, 8)]


def churn(online, M, n=65536, rounds=12, keep=5, seed=3, capacity=64, spread=1):
    heap = Heap(M, capacity, TYPES)
    heap.set_reclaim(online)
    out, errors = heap.stress_churn(n, rounds, keep, seed, spread)
    return heap, out.cpu().numpy().view(np.uint32), errors


@pytest.mark.parametrize("online,M,seed,capacity,rounds", [
    (False, 8192, 3, 64, 12), (True, 8192, 3, 64, 12), (True, 3072, 5, 64, 6), (True, 6144, 7, 32, 6),
    (True, 2600, 9, 64, 4)])
def test_churn_hands_every_slot_out_once(online, M, seed, capacity, rounds):
    # One fifth of the objects are kept (65,536 lanes x rounds / 5) and every
    # wavefront holds a block's worth more while it churns: the smaller heaps
    # leave a few hundred blocks spare, so blocks are freed and taken again by
    # other types as fast as the wavefronts run.
    heap, out, errors = churn(online, M=M, seed=seed, capacity=capacity, rounds=rounds)
    assert errors == 0
    st = heap.stats(raise_sticky=False)
    assert st["oom"] == 0 and st["retry_limit_hit"] == 0 and st["double_free"] == 0
    kept = out[out != C.NULL]
    assert len(np.unique(kept)) == len(kept)                      # I1
    n, rounds = out.shape
    wave = np.arange(n)[:, None] // 64
    types = (wave + np.arange(rounds)[None, :]) % len(TYPES)
    for t in range(len(TYPES)):
        mine = out[(types == t) & (out != C.NULL)]
        assert st["live"][t] == len(mine)
        f0 = heap.field_read(t, 0, torch.tensor(mine.view(np.int32), device="cuda")).cpu().numpy().view(np.uint32)
        assert np.array_equal(f0, mine)                            # nobody else wrote into a kept object
        assert st["allocs"][t] - st["frees"][t] == len(mine)
    # Whether a block empties while online release is on depends on how the
    # wavefronts interleave (a fifth of every wavefront's objects are kept),
    # so the number of releases is not checked here; the test below, which
    # keeps nothing, needs them.
    heap.reclaim()
    assert heap.check() == {}


def test_online_reclaim_reuses_blocks_across_types():
    # 1024 wavefronts, all of them on type r mod 4 in round r, each holding one
    # block at a time: 4 x 1024 blocks are needed if emptied blocks stay with
    # their type until the kernel ends, 1024 if they are freed at once.
    heap, out, errors = churn(False, M=2048, keep=1 << 30, spread=0)
    assert heap.stats(raise_sticky=False)["oom"] == 1
    heap, out, errors = churn(True, M=2048, keep=1 << 30, spread=0)
    st = heap.stats(raise_sticky=False)
    assert errors == 0 and st["oom"] == 0 and st["retry_limit_hit"] == 0
    assert st["online_releases"] >= 2048
    assert (out == C.NULL).all() and st["live"] == [0, 0, 0, 0]
    heap.reclaim()
    assert heap.check() == {}


def test_churn_per_type_capacities_online():
    heap, out, errors = churn(True, M=8192, capacity=0, rounds=8)
    st = heap.stats(raise_sticky=False)
    assert errors == 0 and st["oom"] == 0 and st["retry_limit_hit"] == 0
    kept = out[out != C.NULL]
    assert len(np.unique(kept)) == len(kept) and sum(st["live"]) == len(kept)
    heap.reclaim()
    assert heap.check() == {}


def test_gol_online_equals_oracle():
    rng = np.random.default_rng(4)
    grids = [W.gol_grid(int(s), int(s), seed=400 + i) for i, s in enumerate(rng.integers(5, 120, size=6))]
    gol = apps.GameOfLife(grids)
    gol.heap.set_reclaim(True)
    gol.init()
    gol.step(60, C.DO_PERSISTENT | C.GOL_GRAPH)
    for got, g in zip(gol.read(), grids):
        assert np.array_equal(got, oracle.gol_run(g, 60)[0])
    st = gol.heap.stats()
    assert st["online_releases"] > 0
    gol.heap.reclaim()
    assert gol.heap.check() == {}


def test_micro_online_equals_oracle():
    inp = W.micro_inputs(65536, 10)
    mb = apps.MicroBench(inp, 4096, 64)
    mb.heap.set_reclaim(True)
    mb.heap.set_launch(64, 1)  # split do-all with several blocks per pass
    mb.run()
    res = mb.result()
    ref = oracle.micro_run(inp)
    p = ref.present.astype(bool)
    assert np.array_equal(res.present.astype(bool), p)
    assert np.array_equal(res.x[p].view(np.uint32), ref.x[p].view(np.uint32))
    assert res.stats["allocs"] == [ref.allocs] and res.stats["frees"] == [ref.frees]


def test_traffic_and_sugarscape_online_equal_oracle():
    inp = W.traffic_inputs(50, 200, seed=6)
    sim = apps.Traffic(inp, W.TRAFFIC_RULES)
    sim.heap.set_reclaim(True)
    sim.init()
    sim.step(80, C.DO_PERSISTENT | C.GRAPH)
    assert np.array_equal(sim.read(), oracle.traffic_run(inp.vel, 80, inp.seed, W.TRAFFIC_RULES).vel)
    sug = W.sugar_inputs(48, 500, seed=8)
    s = apps.Sugarscape(sug, W.SUGAR_RULES)
    s.heap.set_reclaim(True)
    s.init()
    s.step(60, C.DO_PERSISTENT | C.GRAPH)
    got = s.read()
    st = oracle.SugarState(sug.side, sug.sugar, sug.cap, sug.occ, sug.a_sugar, sug.a_metab, sug.a_vision,
                           sug.a_age)
    ref = oracle.sugar_run(st, 60, sug.seed, W.SUGAR_RULES)
    assert np.array_equal(got.sugar, ref.sugar) and np.array_equal(got.occ, ref.occ)


@pytest.mark.parametrize("policy", [C.POLICY_BOUNDED, C.POLICY_DENSE])
def test_wator_online_equals_oracle(policy):
    # Many sharks (40 % of the cells) starve within a few steps and empty
    # their blocks, which online release frees inside the kernel and the
    # newborns take again; the sea and the object counts stay the oracle's.
    inp = W.wator_inputs(96, seed=9, fish24=int(0.2 * (1 << 24)), shark24=int(0.4 * (1 << 24)))
    sea = apps.Wator(inp, W.WATOR_RULES)
    for t in range(2):
        sea.heap.set_type_policy(t, policy)
    sea.heap.set_reclaim(True)
    sea.init()
    sea.step(40, C.DO_PERSISTENT | C.GRAPH)
    got = sea.read()
    ref = oracle.wator_run(oracle.WatorState(inp.kind, inp.age, inp.energy), 40, inp.seed, W.WATOR_RULES)
    for f in ("kind", "age", "energy"):
        assert np.array_equal(getattr(got, f), getattr(ref, f)), f
    assert got.stats["live"] == [int((ref.kind == 1).sum()), int((ref.kind == 2).sum())]
    assert got.stats["online_releases"] > 0
    assert sea.heap.check() == {}
    sea.close()
