"""World pools (Game of Life and Sugarscape) driven through the C ABI directly: admission's
argument checks (an occupied or missing slot, side 0, a cell range past the
arena's end or overlapping a resident world) leave the pool untouched, and
worlds admitted flush against the arena's end and into the cells a retired
world left step exactly as the oracle does (the B3/S23 stencil, the Sugarscape
rules with each world's own seed)."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd.serve import Pool  # noqa: E402
from synth import workloads as W  # noqa: E402

ARENA = 2000


def admit(pool, slot, off, grid):
    dev = torch.from_numpy(np.ascontiguousarray(grid, dtype=np.uint8).ravel()).cuda()
    side = grid.shape[0] if grid.size else 0
    rc = pool.lib.dsoar_gol_admit(pool.p, slot, off, side, dev.data_ptr(), pool.heap._s())
    pool.stream.synchronize()
    return rc


def read(pool, slot, side):
    out = torch.empty(side * side, dtype=torch.uint8, device="cuda")
    C.check(pool.lib.dsoar_gol_read_world(pool.p, slot, out.data_ptr(), pool.heap._s()), "dsoar_gol_read_world")
    pool.stream.synchronize()
    return out.cpu().numpy().reshape(side, side)


def step(pool, gens):
    C.check(pool.lib.dsoar_gol_step(pool.p, gens, C.DO_PERSISTENT, pool.heap._s()), "dsoar_gol_step")
    pool.stream.synchronize()


def test_admission_checks_and_reused_cells():
    pool = Pool("gol", 4096, 4, ARENA, graph=False)
    try:
        gA, gB = W.gol_grid(20, 20, seed=1), W.gol_grid(30, 30, seed=2)
        gC, gD = W.gol_grid(10, 10, seed=3), W.gol_grid(10, 10, seed=4)
        assert admit(pool, 0, 0, gA) == C.OK                       # cells [0, 400)
        live0 = pool.heap.stats()["live"]
        assert admit(pool, 1, ARENA - 900 + 1, gB) == C.ERR_INVALID_ARG  # one cell past the end
        assert admit(pool, 0, 1000, gC) == C.ERR_INVALID_ARG       # slot 0 is occupied
        assert admit(pool, 4, 1000, gC) == C.ERR_INVALID_ARG       # only slots 0 .. 3
        assert admit(pool, 2, 395, gC) == C.ERR_INVALID_ARG        # overlaps [0, 400)
        assert admit(pool, 2, 1000, np.zeros((0, 0), np.uint8)) == C.ERR_INVALID_ARG  # side 0
        assert pool.heap.stats()["live"] == live0                  # rejected calls changed nothing
        assert admit(pool, 1, ARENA - 900, gB) == C.OK             # flush against the end
        step(pool, 5)
        assert np.array_equal(read(pool, 0, 20), oracle.gol_run(gA, 5)[0])
        assert np.array_equal(read(pool, 1, 30), oracle.gol_run(gB, 5)[0])
        C.check(pool.lib.dsoar_gol_retire(pool.p, 0, pool.heap._s()), "dsoar_gol_retire")
        assert admit(pool, 0, 0, gC) == C.OK                       # into the retired world's cells
        assert admit(pool, 2, 100, gD) == C.OK
        step(pool, 3)
        assert np.array_equal(read(pool, 1, 30), oracle.gol_run(gB, 8)[0])
        assert np.array_equal(read(pool, 0, 10), oracle.gol_run(gC, 3)[0])
        assert np.array_equal(read(pool, 2, 10), oracle.gol_run(gD, 3)[0])
        assert pool.heap.check() == {}
    finally:
        pool.close()


RULES = W.SUGAR_RULES


def sugar_admit(pool, slot, off, inp):
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in
           (inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab, inp.a_vision, inp.a_age)]
    rc = pool.lib.dsoar_sugar_admit(pool.p, slot, off, inp.side, inp.seed, 0, *[t.data_ptr() for t in dev],
                                    pool.heap._s())
    pool.stream.synchronize()
    return rc


def sugar_check(pool, slot, inp, steps):
    n = inp.side * inp.side
    outs = [torch.empty(n, dtype=dt, device="cuda") for dt in
            (torch.int32, torch.uint8, torch.int32, torch.int32, torch.int32, torch.int32)]
    moves = ctypes.c_uint64()
    C.check(pool.lib.dsoar_sugar_read_world(pool.p, slot, *[t.data_ptr() for t in outs], ctypes.byref(moves),
                                            pool.heap._s()), "dsoar_sugar_read_world")
    pool.stream.synchronize()
    got = [t.cpu().numpy() for t in outs]
    st = oracle.SugarState(inp.side, inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab, inp.a_vision,
                           inp.a_age)
    ref = oracle.sugar_run(st, steps, inp.seed, RULES)
    assert np.array_equal(got[0], ref.sugar) and np.array_equal(got[1], ref.occ)
    m = ref.occ.astype(bool)
    for g, f in zip(got[2:], ("a_sugar", "a_metab", "a_vision", "a_age")):
        assert np.array_equal(g[m], getattr(ref, f)[m])
    assert int(moves.value) == ref.moves


def sugar_step(pool, steps):
    C.check(pool.lib.dsoar_sugar_step(pool.p, steps, C.DO_PERSISTENT, pool.heap._s()), "dsoar_sugar_step")
    pool.stream.synchronize()


def test_sugar_pool_admission_checks_and_reused_cells():
    pool = Pool("sugar", 512, 4, ARENA, rules=RULES, graph=False)
    try:
        iA, iB = W.sugar_inputs(20, 60, seed=5), W.sugar_inputs(30, 150, seed=6)
        iC = W.sugar_inputs(10, 20, seed=7)
        assert sugar_admit(pool, 0, 0, iA) == C.OK                         # cells [0, 400)
        live0 = pool.heap.stats()["live"]
        assert sugar_admit(pool, 1, ARENA - 900 + 1, iB) == C.ERR_INVALID_ARG  # one cell past the end
        assert sugar_admit(pool, 0, 1000, iC) == C.ERR_INVALID_ARG         # slot 0 is occupied
        assert sugar_admit(pool, 4, 1000, iC) == C.ERR_INVALID_ARG         # only slots 0 .. 3
        assert sugar_admit(pool, 2, 399, iC) == C.ERR_INVALID_ARG          # overlaps [0, 400)
        assert pool.heap.stats()["live"] == live0                          # rejected calls changed nothing
        assert sugar_admit(pool, 1, ARENA - 900, iB) == C.OK               # flush against the end
        sugar_step(pool, 4)
        sugar_check(pool, 0, iA, 4)
        sugar_check(pool, 1, iB, 4)
        C.check(pool.lib.dsoar_sugar_retire(pool.p, 0, pool.heap._s()), "dsoar_sugar_retire")
        assert sugar_admit(pool, 0, 50, iC) == C.OK                        # inside the retired world's cells
        sugar_step(pool, 3)
        sugar_check(pool, 1, iB, 7)
        sugar_check(pool, 0, iC, 3)
        assert pool.heap.check() == {}
    finally:
        pool.close()
