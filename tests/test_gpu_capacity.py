"""Per-type block capacities (Sec. 2 byte-size rule, heap capacity 0): the
layout's capacities equal the oracle's; mixed-capacity heaps keep every
invariant under churn and the do-all (64 / c blocks per wavefront) visits each
live object exactly once; Game of Life with Cells at 64 and Alive/Candidate at
16 slots equals the oracle."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd import apps, batch  # noqa: E402
from paper_1809_07444_amd.heap import Heap  # noqa: E402
from synth import workloads as W  # noqa: E402

TYPE_SETS = [
    [(4,), (4, 4, 4), (8, 8, 8), (8, 8, 8, 8)],          # 4, 12, 24, 32 bytes
    [(4, 4), (4, 4, 4), (4, 4, 4)],                      # the Game of Life types
    [(8,), (4,), (8, 8, 8, 8, 8, 8, 8, 8)],              # 8, 4, 64 bytes
]


@pytest.mark.parametrize("types", TYPE_SETS)
def test_layout_capacities_match_oracle(types):
    heap = Heap(256, 0, types)
    sizes = [sum(t) for t in types]
    assert heap.type_capacity == [oracle.type_capacity(sizes, t) for t in range(len(types))]
    L = heap.layout()
    assert L.block_stride >= max(c * s for c, s in zip(heap.type_capacity, sizes))


@pytest.mark.parametrize("wg,per_cu", [(256, 8), (64, 1)])
def test_mixed_capacity_churn_and_visits(wg, per_cu):
    types = TYPE_SETS[0]
    rng = np.random.default_rng(17 + wg)
    M = 1024
    heap = Heap(M, 0, types)
    heap.set_launch(wg, per_cu)
    caps = heap.type_capacity
    assert caps == [64, 16, 8, 8]
    live = {}
    for rnd in range(5):
        for t in range(len(types)):
            n = int(rng.integers(1, 2500 // (65 - caps[t]) + 200))
            h = heap.alloc_n(t, n).cpu().numpy().view(np.uint32)
            h = h[h != C.NULL]
            assert ((h & 63) < caps[t]).all()
            for x in h.tolist():
                assert x not in live
                live[x] = t
        keys = np.array(sorted(live), dtype=np.uint32)
        kill = keys[rng.random(len(keys)) < 0.45]
        heap.free_n(torch.tensor(kill.view(np.int32), device="cuda"))
        for x in kill.tolist():
            del live[x]
        st = heap.stats()
        for t in range(len(types)):
            n_t = sum(1 for v in live.values() if v == t)
            assert st["live"][t] == n_t == st["allocs"][t] - st["frees"][t]
            assert st["allocated_blocks"][t] >= -(-n_t // caps[t])
            counts = heap.visit_counts(t).cpu().numpy()
            exp = np.zeros(M * 64, dtype=np.int32)
            exp[[x for x, v in live.items() if v == t]] = 1
            assert np.array_equal(counts, exp)
        assert heap.check() == {}


@pytest.mark.parametrize("seed", [1, 2])
def test_gol_per_type_capacity_equals_oracle(seed):
    rng = np.random.default_rng(seed)
    sides = rng.integers(3, 90, size=5)
    grids = [W.gol_grid(int(s), int(s), seed=seed * 100 + i) for i, s in enumerate(sides)]
    gol = apps.GameOfLife(grids, capacity=0)
    assert gol.heap.type_capacity == [64, 16, 16]
    gol.init()
    gol.step(40, C.DO_PERSISTENT | C.GOL_GRAPH)
    for got, g in zip(gol.read(), grids):
        assert np.array_equal(got, oracle.gol_run(g, 40)[0])
    assert gol.heap.check() == {}


def test_gol_full_size_per_type_capacity():
    # 1024 x 1024 torus, Bernoulli(0.1), 200 generations, Alive/Candidate at 32 slots.
    g0 = W.gol_grid(1024, 1024)
    gol = apps.GameOfLife([g0], capacity=0)
    gol.init()
    gol.step(200, C.DO_PERSISTENT | C.GOL_GRAPH)
    assert np.array_equal(gol.read()[0], oracle.gol_run(g0, 200)[0])
    assert gol.heap.check() == {}


def test_batched_per_type_capacity_config():
    inp = W.batch_inputs(16, 30, lo=8, hi=80, seed=9)
    b = batch.BatchedGol(inp.grids, batch.TuneConfig(0, 256, 4, batch.NEVER))
    b.run(30)
    for got, g in zip(b.read(), inp.grids):
        assert np.array_equal(got, oracle.gol_run(g, 30)[0])
    assert b.gol.heap.check() == {}
