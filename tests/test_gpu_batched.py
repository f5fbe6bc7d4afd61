"""Many Game-of-Life worlds in one heap (persistent do-alls, graph replay)
against the oracle per world, across autotuner configurations, and against
the per-world plain baseline."""
import hashlib
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import batch  # noqa: E402
from synth import workloads as W  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gol_batched_256w_100g_seed24301.json")


def small_batch(seed=3, n=24, lo=8, hi=96):
    inp = W.batch_inputs(n, 40, lo=lo, hi=hi, seed=seed)
    return inp.grids


def oracle_finals(grids, gens):
    return [oracle.gol_run(g, gens)[0] for g in grids]


H, LO, X = batch.C.SEARCH_HASHED, batch.C.SEARCH_LOWEST, batch.C.SEARCH_XCD


@pytest.mark.parametrize("cfg", [batch.TuneConfig(64, 256, 8, 0), batch.TuneConfig(32, 1024, 2, 0),
                                 batch.TuneConfig(64, 64, 16, batch.NEVER), batch.TuneConfig(32, 256, 4, batch.NEVER),
                                 batch.TuneConfig(64, 256, 8, 0, 32, X), batch.TuneConfig(32, 1024, 2, 0, 32, H),
                                 batch.TuneConfig(0, 256, 4, batch.NEVER, 32, LO),
                                 batch.TuneConfig(64, 256, 8, 0, 64, LO), batch.TuneConfig(0, 64, 16, 0, 64, X)])
def test_batched_matches_oracle_for_every_config(cfg):
    grids = small_batch()
    b = batch.BatchedGol(grids, cfg)
    b.run(40)
    got = b.read()
    for a, e in zip(got, oracle_finals(grids, 40)):
        assert np.array_equal(a, e)
    assert b.gol.heap.check() == {}


def test_plain_matches_batched():
    grids = small_batch(seed=5, n=10)
    p = batch.PlainGol(grids)
    p.run(25)
    s = batch.PlainGol(grids[:3], sync=True)
    s.run(25)
    b = batch.BatchedGol(grids)
    b.run(25)
    exp = oracle_finals(grids, 25)
    for a, c, e in zip(p.read(), b.read(), exp):
        assert np.array_equal(a, e) and np.array_equal(c, e)
    for a, e in zip(s.read(), exp[:3]):
        assert np.array_equal(a, e)
    assert p.stats()["allocs"] == b.stats()["allocs"]


def test_autotune_small_space(tmp_path):
    grids = small_batch(seed=7, n=8)
    space = {"capacity": [64, 32], "bitmap_width": [64, 32], "wg_threads": [256], "wgs_per_cu": [4],
             "bulk_min": [0], "search": [H, X]}
    best, table = batch.autotune(grids, 5, space, cache_path=str(tmp_path / "tune.json"))
    assert len(table) == 8 and best.capacity in (64, 32) and best.bitmap_width in (64, 32)
    assert {r["config"]["bitmap_width"] for r in table} == {64, 32}
    best2, table2 = batch.autotune(grids, 5, space, cache_path=str(tmp_path / "tune.json"))
    assert best2 == best and table2 == table           # served from the cache


def test_full_config_256_worlds_100_generations():
    # 256 worlds, sides log-uniform in 64..1024 (48.2 M cells), Bernoulli(0.1),
    # 100 generations, one heap, graph replay; stored oracle digests per world.
    ref = json.load(open(GOLDEN))
    inp = W.batch_inputs(256, 100)
    assert inp.sides.tolist() == [w["side"] for w in ref["worlds"]]
    b = batch.BatchedGol(inp.grids)
    b.run(100)
    got = b.read()
    for a, w in zip(got, ref["worlds"]):
        assert hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint8).tobytes()).hexdigest() == w["sha256"]
    st = b.stats()
    assert st["allocs"][2] == sum(w["candidates"] for w in ref["worlds"])
    assert st["frees"][1] == sum(w["deaths"] for w in ref["worlds"])
    assert st["allocs"][1] == sum(w["initial_population"] + w["births"] for w in ref["worlds"])
    assert st["live"][1] == sum(w["population"] for w in ref["worlds"])
    # and the smallest worlds against the oracle directly
    small = np.argsort(inp.sides)[:4]
    for i in small:
        assert np.array_equal(got[i], oracle.gol_run(inp.grids[i], 100)[0])
