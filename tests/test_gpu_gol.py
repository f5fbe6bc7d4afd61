"""Game of Life as objects on the device against the oracle's dense B3/S23
torus: exact final grids, and exact object churn (every Candidate is one
dead cell next to a live one; births and deaths are the oracle's)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd import apps  # noqa: E402
from synth import workloads as W  # noqa: E402


def expected_counts(grids, gens):
    allocs = [0, 0, 0]
    frees = [0, 0, 0]
    finals = []
    for g in grids:
        final, c = oracle.gol_run(g, gens)
        finals.append(final)
        allocs[0] += g.size
        allocs[1] += int(g.astype(bool).sum()) + int(c[:, 1].sum())
        frees[1] += int(c[:, 2].sum())
        allocs[2] += int(c[:, 0].sum())
        frees[2] += int(c[:, 0].sum())
    return finals, allocs, frees


def run_and_compare(grids, gens, flags=C.DO_PERSISTENT, capacity=64, split=None, cand_policy=None):
    gol = apps.GameOfLife(grids, capacity=capacity)
    if cand_policy is not None:
        gol.heap.set_type_policy(apps.GOL_CAND, cand_policy)
    gol.init()
    if split:
        for k in split:
            gol.step(k, flags)
    else:
        gol.step(gens, flags)
    got = gol.read()
    finals, allocs, frees = expected_counts(grids, gens)
    for a, b in zip(got, finals):
        assert np.array_equal(a, b)
    st = gol.heap.stats()
    assert st["allocs"] == allocs and st["frees"] == frees
    assert st["live"] == [gol.total, int(sum(f.sum() for f in finals)), 0]
    assert gol.heap.check() == {}
    return gol


def grid_with(n, cells):
    g = np.zeros((n, n), np.uint8)
    for x, y in cells:
        g[y % n, x % n] = 1
    return g


def test_glider_returns_after_full_lap():
    glider = [(1, 0), (2, 1), (0, 2), (1, 2), (2, 2)]
    g0 = grid_with(16, glider)
    gol = run_and_compare([g0], 64)
    assert np.array_equal(gol.read()[0], g0)


def test_still_life_blinker_and_empty_worlds_together():
    worlds = [grid_with(8, [(1, 1), (2, 1), (1, 2), (2, 2)]),        # block
              grid_with(5, [(2, 1), (2, 2), (2, 3)]),                # blinker
              np.zeros((7, 7), np.uint8),                             # empty
              np.ones((1, 1), np.uint8), np.ones((2, 2), np.uint8)]  # degenerate tori
    run_and_compare(worlds, 7)


@pytest.mark.parametrize("seed,capacity", [(1, 64), (2, 32), (3, 64), (4, 32), (5, 64)])
def test_random_small_worlds(seed, capacity):
    rng = np.random.default_rng(seed)
    sides = rng.integers(3, 70, size=6)
    grids = [W.gol_grid(int(s), int(s), seed=seed * 100 + i, threshold24=int(rng.integers(1, 1 << 23)))
             for i, s in enumerate(sides)]
    run_and_compare(grids, 50, capacity=capacity)


@pytest.mark.parametrize("flags", [C.DO_PLAIN, C.DO_PERSISTENT | C.GOL_GRAPH])
def test_modes_agree_medium(flags):
    grids = [W.gol_grid(200, 200, seed=11), W.gol_grid(97, 97, seed=12)]
    run_and_compare(grids, 40, flags=flags, split=[1, 13, 26])


@pytest.mark.parametrize("policy", [C.POLICY_DENSE, C.POLICY_FRESH])
def test_candidate_policies_agree(policy):
    # Candidates from active blocks first (dense) or from blocks of their own
    # (fresh): placement differs, grids and object counts do not.
    grids = [W.gol_grid(256, 256, seed=21), W.gol_grid(61, 61, seed=22)]
    run_and_compare(grids, 60, flags=C.DO_PERSISTENT | C.GOL_GRAPH, cand_policy=policy)


def test_type_policy_validates():
    gol = apps.GameOfLife([W.gol_grid(16, 16, seed=3)])
    with pytest.raises(Exception):
        gol.heap.set_type_policy(3, C.POLICY_FRESH)  # three types: 0, 1, 2
    with pytest.raises(Exception):
        gol.heap.set_type_policy(0, 3)


def test_full_config_1024_200_generations():
    # 1024 x 1024 torus, Bernoulli(0.1) alive, 200 generations (graph replay).
    g0 = W.gol_grid(1024, 1024)
    run_and_compare([g0], 200, flags=C.DO_PERSISTENT | C.GOL_GRAPH)


@pytest.mark.parametrize("shift", [1, 8])
def test_wide_init_from_an_unaligned_grid(shift):
    # A world set of 2^22 cells or more is created 64 cells per lane, with
    # 16-byte grid loads where the caller's grid allows them: a grid that
    # starts 1 or 8 bytes past an aligned address takes the byte loads and
    # gives the same world.  Two worlds whose boundary falls inside a lane's
    # 64 cells check the per-cell world lookup.
    g0 = W.gol_grid(2048, 2048, seed=9)
    g1 = W.gol_grid(65, 65, seed=10)
    gol = apps.GameOfLife([g1, g0])
    flat = np.concatenate([g1.reshape(-1), g0.reshape(-1)])
    buf = torch.zeros(flat.size + shift, dtype=torch.uint8, device="cuda")
    buf[shift:] = torch.from_numpy(flat).cuda()
    gol.heap.reset()
    C.check(gol.lib.dsoar_gol_init(gol.g, buf.data_ptr() + shift, gol.heap._s()), "dsoar_gol_init")
    gol.step(12, C.DO_PERSISTENT)
    finals, allocs, frees = expected_counts([g1, g0], 12)
    for a, b in zip(gol.read(), finals):
        assert np.array_equal(a, b)
    st = gol.heap.stats()
    assert st["allocs"] == allocs and st["frees"] == frees
    assert gol.heap.check() == {}


@pytest.mark.parametrize("capacity,flags", [(64, C.DO_PERSISTENT), (64, C.DO_PERSISTENT | C.GOL_GRAPH),
                                            (32, C.DO_PERSISTENT)])
def test_paired_passes_on_a_small_grid(capacity, flags):
    # With one 64-thread workgroup per CU the persistent do-all has 256
    # wavefronts, so lists of 512 blocks or more go two entries per pass
    # (the pair form, one allocation request for both blocks) and shorter
    # ones one entry per pass: about 1,600 Alive and 2,000 Candidate blocks
    # here, and a ragged last pair.  Capacity 32 takes the per-lane form.
    grids = [W.gol_grid(1024, 1024, seed=31), W.gol_grid(300, 300, seed=32)]
    gol = apps.GameOfLife(grids, capacity=capacity)
    gol.heap.set_launch(64, 1)
    gol.init()
    gol.step(40, flags)
    finals, allocs, frees = expected_counts(grids, 40)
    for a, b in zip(gol.read(), finals):
        assert np.array_equal(a, b)
    st = gol.heap.stats()
    assert st["allocs"] == allocs and st["frees"] == frees
    assert gol.heap.check() == {}
