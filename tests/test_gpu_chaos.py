"""The heap under the stress build: libdsoar_chaos.so is the same library
compiled with DSOAR_CHAOS, which makes a wavefront pause (about one time in
four, for up to about 12 us) inside the race windows of the allocator: between
reading an active block's object bitmap and reserving in it, between taking
free blocks and publishing them, between publishing and setting their
allocated / active bits, between a container's update and its nested bit one
level up, between a full block's delete and its return to active, and between
the steps of an online release.  Other wavefronts' atomics then land inside
those windows far more often than in the release build.  Every outcome must
still be the exact one: the bitmap storms' results and final words, slots
handed out once, live counts, the invariants at quiescence, and the oracle's
results for the applications."""
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd import apps  # noqa: E402
from paper_1809_07444_amd.heap import DeviceBitmap, Heap  # noqa: E402
from synth import workloads as W  # noqa: E402


@pytest.fixture(autouse=True)
def chaos():
    with C.using("chaos") as lib:
        assert os.path.basename(lib._name) == "libdsoar_chaos.so"
        yield lib


def ops(kinds, poss):
    return torch.tensor(np.stack([kinds, poss], axis=1).astype(np.int32), device="cuda")


def level_words(bm):
    return [w.cpu().numpy().view(np.uint64 if bm.width == 64 else np.uint32) for w in bm.level_words()]


@pytest.mark.parametrize("width", [64, 32])
@pytest.mark.parametrize("nbits,seed", [(4096, 11), (64 ** 3 + 17, 12)])
def test_bitmap_storm_exact_under_chaos(nbits, seed, width):
    # One try_set or try_clear per position, all at once, from a 30 % start:
    # the results and every level's words equal the sequential model's.
    rng = np.random.default_rng(seed)
    init = rng.random(nbits) < 0.3
    bm = DeviceBitmap(nbits, width=width)
    pos0 = np.nonzero(init)[0]
    assert (bm.run(ops(np.full(len(pos0), C.BM_TRY_SET), pos0)).cpu().numpy() == 1).all()
    n = min(nbits, 20000)
    pos = rng.permutation(nbits)[:n]
    kinds = rng.integers(0, 2, size=n)
    res = bm.run(ops(kinds, pos)).cpu().numpy()
    assert np.array_equal(res, np.where(kinds == 0, ~init[pos], init[pos]).astype(np.int32))
    final = init.copy()
    final[pos[kinds == 0]] = True
    final[pos[kinds == 1]] = False
    ref = oracle.Bitmap(nbits, width)
    for p in np.nonzero(final)[0]:
        ref.try_set(int(p))
    lv = level_words(bm)
    assert len(lv) == ref.nlevels
    for lvl, w in enumerate(lv):
        assert [int(x) for x in w] == [int(x) for x in ref.words(lvl)], lvl


@pytest.mark.parametrize("width", [64, 32])
def test_bitmap_set_clear_pairs_and_drain_under_chaos(width):
    # set and clear of the same clear bit meet (clear retries until the set
    # lands), then find_clear drains a full bitmap handing each bit out once.
    nbits = 8192
    bm = DeviceBitmap(nbits, width=width)
    pos = np.arange(0, nbits, 8)
    kinds = np.concatenate([np.full(len(pos), C.BM_CLEAR), np.full(len(pos), C.BM_SET)])
    assert (bm.run(ops(kinds, np.concatenate([pos, pos]))).cpu().numpy() == 0).all()
    assert all(int(w.abs().sum()) == 0 for w in bm.level_words())
    full = DeviceBitmap(5000, all_set=True, width=width)
    n = 5100
    starts = torch.tensor(np.random.default_rng(3).integers(0, 2 ** 31, size=n).astype(np.int32), device="cuda")
    res = full.run(ops(np.full(n, C.BM_FIND_CLEAR), np.zeros(n, np.int64)), starts).cpu().numpy()
    got = res[res >= 0]
    assert len(got) == 5000 and len(set(got.tolist())) == 5000
    assert all(int(w.abs().sum()) == 0 for w in full.level_words())


@pytest.mark.parametrize("online,M,capacity,rounds", [(False, 8192, 64, 6), (True, 3072, 64, 6),
                                                      (True, 6144, 32, 4)])
def test_reclaim_churn_hands_every_slot_out_once_under_chaos(online, M, capacity, rounds):
    types = [(4,), (4, 4), (4, 4, 4), (4, 8)]
    heap = Heap(M, capacity, types)
    heap.set_reclaim(online)
    out, errors = heap.stress_churn(65536, rounds, 5, 21, 1)
    out = out.cpu().numpy().view(np.uint32)
    assert errors == 0
    st = heap.stats(raise_sticky=False)
    assert st["oom"] == 0 and st["retry_limit_hit"] == 0 and st["double_free"] == 0
    kept = out[out != C.NULL]
    assert len(np.unique(kept)) == len(kept)
    n, r = out.shape
    tmap = ((np.arange(n)[:, None] // 64) + np.arange(r)[None, :]) % len(types)
    for t in range(len(types)):
        mine = out[(tmap == t) & (out != C.NULL)]
        assert st["live"][t] == len(mine) == st["allocs"][t] - st["frees"][t]
        f0 = heap.field_read(t, 0, torch.tensor(mine.view(np.int32), device="cuda")).cpu().numpy().view(np.uint32)
        assert np.array_equal(f0, mine)
    heap.reclaim()
    assert heap.check() == {}


@pytest.mark.parametrize("cap,width", [(64, 64), (32, 32)])
def test_alloc_free_rounds_under_chaos(cap, width):
    rng = np.random.default_rng(cap)
    heap = Heap(512, cap, [(4, 8)] * 2, bitmap_width=width)
    live = {}
    for _ in range(5):
        for t in range(2):
            h = heap.alloc_n(t, int(rng.integers(1, 4000))).cpu().numpy().view(np.uint32)
            for x in h[h != C.NULL].tolist():
                assert x not in live
                live[x] = t
        keys = np.array(sorted(live), dtype=np.uint32)
        kill = keys[rng.random(len(keys)) < 0.5]
        heap.free_n(torch.tensor(kill.view(np.int32), device="cuda"))
        for x in kill.tolist():
            del live[x]
        st = heap.stats()
        for t in range(2):
            assert st["live"][t] == sum(1 for v in live.values() if v == t) == st["allocs"][t] - st["frees"][t]
            counts = heap.visit_counts(t).cpu().numpy()
            exp = np.zeros(512 * 64, dtype=np.int32)
            exp[[x for x, v in live.items() if v == t]] = 1
            assert np.array_equal(counts, exp)
        assert heap.check() == {}


def gol_expected(grids, gens):
    allocs, frees, finals = [0, 0, 0], [0, 0, 0], []
    for g in grids:
        final, c = oracle.gol_run(g, gens)
        finals.append(final)
        allocs[0] += g.size
        allocs[1] += int(g.astype(bool).sum()) + int(c[:, 1].sum())
        frees[1] += int(c[:, 2].sum())
        allocs[2] += int(c[:, 0].sum())
        frees[2] += int(c[:, 0].sum())
    return finals, allocs, frees


@pytest.mark.parametrize("capacity,width,online,flags", [
    (64, 64, False, C.DO_PERSISTENT | C.GRAPH), (32, 32, False, C.DO_PLAIN), (64, 32, True, C.DO_PERSISTENT)])
def test_game_of_life_equals_oracle_under_chaos(capacity, width, online, flags):
    grids = [W.gol_grid(s, s, seed=40 + s) for s in (37, 64, 90)]
    gol = apps.GameOfLife(grids, capacity=capacity, bitmap_width=width)
    gol.heap.set_reclaim(online)
    gol.init()
    gol.step(25, flags)
    finals, allocs, frees = gol_expected(grids, 25)
    for a, b in zip(gol.read(), finals):
        assert np.array_equal(a, b)
    st = gol.heap.stats()
    assert st["allocs"] == allocs and st["frees"] == frees
    assert gol.heap.check() == {}


def test_game_of_life_paired_passes_under_chaos():
    # 256 persistent wavefronts: the Alive and Candidate lists of a 1024^2
    # world go two blocks per pass.
    grids = [W.gol_grid(1024, 1024, seed=33)]
    gol = apps.GameOfLife(grids)
    gol.heap.set_launch(64, 1)
    gol.init()
    gol.step(20, C.DO_PERSISTENT)
    finals, allocs, frees = gol_expected(grids, 20)
    assert np.array_equal(gol.read()[0], finals[0])
    st = gol.heap.stats()
    assert st["allocs"] == allocs and st["frees"] == frees
    assert gol.heap.check() == {}


@pytest.mark.parametrize("cap,flags", [(64, C.DO_PERSISTENT), (32, C.DO_PLAIN)])
def test_microbenchmark_equals_oracle_under_chaos(cap, flags):
    inp = W.micro_inputs(20000, 4, seed=17)
    res = apps.micro_run(inp, num_blocks=1024, capacity=cap, flags=flags)
    ref = oracle.micro_run(inp)
    p = ref.present.astype(bool)
    assert np.array_equal(res.present.astype(bool), p)
    assert np.array_equal(res.x[p].view(np.uint32), ref.x[p].view(np.uint32))
    assert res.stats["allocs"] == [ref.allocs] and res.stats["frees"] == [ref.frees]


@pytest.mark.parametrize("online", [False, True])
def test_sugarscape_equals_oracle_under_chaos(online):
    # Births (new agents of the agents' own type) and deaths in the same
    # steps, on a crowded 64 x 64 torus.
    inp = W.sugar_inputs(64, 1500, seed=13)
    rules = W.SUGAR_RULES
    sim = apps.Sugarscape(inp, rules)
    sim.heap.set_reclaim(online)
    sim.init()
    sim.step(25, C.DO_PERSISTENT | C.GRAPH)
    ref = oracle.sugar_run(oracle.SugarState(inp.side, inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab,
                                             inp.a_vision, inp.a_age), 25, inp.seed, rules)
    got = sim.read()
    assert np.array_equal(got.sugar, ref.sugar) and np.array_equal(got.occ, ref.occ)
    m = ref.occ.astype(bool)
    for f in ("a_sugar", "a_metab", "a_vision", "a_age"):
        assert np.array_equal(getattr(got, f)[m], getattr(ref, f)[m]), f
    n0 = int(inp.occ.sum())
    assert got.stats["allocs"] == [n0 + ref.births] and got.stats["frees"] == [ref.deaths]
    assert sim.heap.check() == {}


@pytest.mark.parametrize("online", [False, True])
def test_wator_equals_oracle_under_chaos(online):
    # Sharks that starve (delete themselves) and breed (new sharks) in the
    # same do-all, fish eaten and born: the pattern of the settle ordering.
    inp = W.wator_inputs(128, seed=14)
    rules = W.WATOR_RULES
    sea = apps.Wator(inp, rules)
    sea.heap.set_reclaim(online)
    sea.init()
    sea.step(30, C.DO_PERSISTENT | C.GRAPH)
    ref = oracle.wator_run(oracle.WatorState(inp.kind, inp.age, inp.energy), 30, inp.seed, rules)
    got = sea.read()
    for f in ("kind", "age", "energy"):
        assert np.array_equal(getattr(got, f), getattr(ref, f)), f
    f0, s0 = int((inp.kind == 1).sum()), int((inp.kind == 2).sum())
    assert got.stats["allocs"] == [f0 + ref.fish_born, s0 + ref.sharks_born]
    assert got.stats["frees"] == [ref.fish_eaten, ref.sharks_starved]
    assert sea.heap.check() == {}
    sea.close()


def test_traffic_equals_oracle_under_chaos():
    # Cars enter (new, into nearly full active blocks) and leave (delete).
    inp = W.traffic_inputs(37, 211, seed=15)
    rules = W.TRAFFIC_RULES
    sim = apps.Traffic(inp, rules)
    sim.init()
    sim.step(60, C.DO_PERSISTENT | C.GRAPH)
    r = oracle.traffic_run(inp.vel, 60, inp.seed, rules)
    assert np.array_equal(sim.read(), r.vel)
    st = sim.heap.stats()
    assert st["allocs"] == [int((inp.vel >= 0).sum()) + r.entries] and st["frees"] == [r.exits]
    assert sim.heap.check() == {}
