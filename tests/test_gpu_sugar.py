"""Sugarscape-style agents on the device against the oracle's sequential
rules: exact grids, agents canonicalised by cell, and exact birth, death and
move counts."""
import hashlib
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd import apps  # noqa: E402
from synth import workloads as W  # noqa: E402

RULES = W.SUGAR_RULES
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sugarscape_2048_1048576a_500s_seed24301.json")


def to_state(inp):
    return oracle.SugarState(inp.side, inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab, inp.a_vision,
                             inp.a_age)


def compare(got, ref, n_init):
    assert np.array_equal(got.sugar, ref.sugar)
    assert np.array_equal(got.occ, ref.occ)
    m = ref.occ.astype(bool)
    for f in ("a_sugar", "a_metab", "a_vision", "a_age"):
        assert np.array_equal(getattr(got, f)[m], getattr(ref, f)[m]), f
    st = got.stats
    assert st["status"] == C.OK
    assert st["allocs"] == [n_init + ref.births] and st["frees"] == [ref.deaths]
    assert st["live"] == [int(m.sum())]
    assert got.moves == ref.moves


def hand_case():
    # 5x5: conflict over cell 12 (west neighbour 11 wins), a fertile rich
    # agent that gives birth, and one that dies of age.
    inp = W.sugar_inputs(5, 0, seed=77)
    inp.cap[:] = 0
    inp.sugar[:] = 0
    inp.cap[12] = inp.sugar[12] = 4
    for c, (s, m, v, a) in {11: (6, 2, 1, 3), 13: (6, 2, 1, 3), 2: (30, 1, 1, 20),
                            20: (50, 1, 1, RULES["max_age"] - 1)}.items():
        inp.occ[c] = 1
        inp.a_sugar[c], inp.a_metab[c], inp.a_vision[c], inp.a_age[c] = s, m, v, a
    return inp


@pytest.mark.parametrize("flags", [C.DO_PERSISTENT, C.DO_PLAIN, C.DO_PERSISTENT | C.GRAPH])
def test_hand_case(flags):
    inp = hand_case()
    sim = apps.Sugarscape(inp, RULES)
    sim.init()
    sim.step(3, flags)
    ref = oracle.sugar_run(to_state(inp), 3, inp.seed, RULES)
    compare(sim.read(), ref, int(inp.occ.sum()))


@pytest.mark.parametrize("side,agents,seed,cap", [(16, 40, 1, 64), (33, 300, 2, 32), (64, 1000, 3, 64),
                                                   (64, 3000, 4, 32), (1, 1, 5, 64), (2, 3, 6, 64),
                                                   (8, 0, 7, 64)])  # no agents: regrowth only
def test_random_worlds(side, agents, seed, cap):
    inp = W.sugar_inputs(side, agents, seed=seed)
    sim = apps.Sugarscape(inp, RULES, capacity=cap)
    sim.init()
    ref = to_state(inp)
    done = 0
    for k in (1, 9, 30):
        sim.step(k, C.DO_PERSISTENT | C.GRAPH)
        ref = oracle.sugar_run(ref, k, inp.seed, RULES, step0=done)
        done += k
        compare(sim.read(), ref, int(inp.occ.sum()))
    assert sim.heap.check() == {}


def test_sugar_at_the_top_of_its_byte():
    # A cell keeps its sugar in seven bits beside the occupancy bit: capacities
    # and sugar of 100..127 (the largest the grid holds), regrowing and eaten
    # every step, still give the oracle's world.
    import dataclasses
    inp = W.sugar_inputs(48, 500, seed=11)
    cap = np.random.default_rng(11).integers(100, 128, size=inp.cap.shape).astype(inp.cap.dtype)
    inp = dataclasses.replace(inp, cap=cap, sugar=cap.copy())
    sim = apps.Sugarscape(inp, RULES)
    sim.init()
    ref = to_state(inp)
    done = 0
    for k in (1, 9, 30):
        sim.step(k, C.DO_PERSISTENT | C.GRAPH)
        ref = oracle.sugar_run(ref, k, inp.seed, RULES, step0=done)
        done += k
        compare(sim.read(), ref, int(inp.occ.sum()))
    assert sim.heap.check() == {}


def test_full_config_2048_1M_agents_500_steps():
    # 2048 x 2048 torus, 2^20 agents, 500 steps; stored oracle digests every 100 steps.
    ref = json.load(open(GOLDEN))
    inp = W.sugar_inputs(2048, 1 << 20)
    sim = apps.Sugarscape(inp, RULES)
    sim.init()
    done = 0
    for cp in ref["checkpoints"]:
        sim.step(cp["step"] - done, C.DO_PERSISTENT | C.GRAPH)
        done = cp["step"]
        got = sim.read()
        m = got.occ.astype(bool)
        assert int(m.sum()) == cp["agents"]
        assert hashlib.sha256(np.ascontiguousarray(got.sugar).tobytes()).hexdigest() == cp["sugar_grid_sha256"]
        assert hashlib.sha256(np.ascontiguousarray(got.occ).tobytes()).hexdigest() == cp["occ_sha256"]
        agents = np.stack([got.a_sugar, got.a_metab, got.a_vision, got.a_age]).astype(np.int32)
        assert hashlib.sha256(np.ascontiguousarray(agents).tobytes()).hexdigest() == cp["agents_sha256"]
        assert got.stats["allocs"] == [(1 << 20) + cp["births"]] and got.stats["frees"] == [cp["deaths"]]
        assert got.moves == cp["moves"]


@pytest.mark.parametrize("field,value", [("cap", 200), ("sugar", 128), ("sugar", -1), ("cap", -5)])
def test_c_abi_refuses_sugar_outside_a_cells_byte(field, value):
    # Straight through the C ABI (the Python wrapper refuses such input
    # itself): the library returns INVALID_ARG, creates no agent and leaves
    # the world unadmitted.
    import ctypes
    import torch
    inp = W.sugar_inputs(16, 20, seed=3)
    sim = apps.Sugarscape(inp, RULES)
    bad = [t.clone() for t in sim.inputs]
    k = 0 if field == "sugar" else 1
    bad[k][37] = value
    sim.heap.reset()
    rc = sim.lib.dsoar_sugar_init(sim.s, *[t.data_ptr() for t in bad], 0, sim.heap._s())
    assert rc == C.ERR_INVALID_ARG
    st = sim.heap.stats(raise_sticky=False)
    assert st["allocs"] == [0] and st["live"] == [0]
    assert sim.lib.dsoar_sugar_read(sim.s, *[t.data_ptr() for t in sim.out], None, sim.heap._s()) == \
        C.ERR_INVALID_ARG  # slot 0 was never admitted
    # The same world with the value in range is admitted and runs.
    sim.init()
    sim.step(3, C.DO_PERSISTENT)
    ref = oracle.sugar_run(to_state(inp), 3, inp.seed, RULES)
    compare(sim.read(), ref, int(inp.occ.sum()))
    torch.cuda.synchronize()
