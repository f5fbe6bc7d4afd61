"""Wa-Tor on the device against the oracle: the sea (kind, age, energy per
cell) equal after every checked step, and the object churn exact (fish and
shark objects created = initial + born, deleted = eaten / starved)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd import apps  # noqa: E402
from synth import workloads as W  # noqa: E402

GRAPH = C.DO_PERSISTENT | C.GRAPH
RULES = W.WATOR_RULES


def check(inp, split, flags=C.DO_PERSISTENT, capacity=64, rules=RULES):
    sea = apps.Wator(inp, rules, capacity=capacity)
    sea.init()
    ref = oracle.WatorState(inp.kind, inp.age, inp.energy)
    f0, s0 = int((inp.kind == 1).sum()), int((inp.kind == 2).sum())
    done = 0
    for k in split:
        sea.step(k, flags)
        ref = oracle.wator_run(ref, k, inp.seed, rules, step0=done)
        done += k
        got = sea.read()
        for f in ("kind", "age", "energy"):
            assert np.array_equal(getattr(got, f), getattr(ref, f)), f"{f} differs after {done} steps"
        st = got.stats
        assert st["allocs"] == [f0 + ref.fish_born, s0 + ref.sharks_born]
        assert st["frees"] == [ref.fish_eaten, ref.sharks_starved]
        assert st["live"] == [int((ref.kind == 1).sum()), int((ref.kind == 2).sum())]
    assert sea.heap.check() == {}
    sea.close()
    return ref


def inputs_of(side, cells, seed=5):
    k = np.zeros((side, side), np.int32)
    a = np.zeros((side, side), np.int32)
    e = np.zeros((side, side), np.int32)
    for (x, y), (kk, aa, ee) in cells.items():
        k[y, x], a[y, x], e[y, x] = kk, aa, ee
    return W.WatorInputs(side, seed, k, a, e)


def test_hand_cases():
    check(inputs_of(7, {(3, 3): (1, 0, 0)}), [1, 1, 1, 3])                      # lone fish breeds
    check(inputs_of(2, {(x, y): (1, 5, 0) for x in range(2) for y in range(2)}), [4])   # boxed in
    check(inputs_of(3, {(x, y): (1, 2, 0) for x in range(3) for y in range(3) if (x, y) != (1, 1)}), [1])
    check(inputs_of(2, {(0, 0): (2, 0, 1), (1, 0): (1, 0, 0), (0, 1): (1, 0, 0), (1, 1): (1, 0, 0)}), [1])
    check(inputs_of(5, {(2, 2): (2, 0, 3)}), [1, 1, 1])                          # starves
    check(inputs_of(1, {(0, 0): (2, 0, 2)}), [3])                                # 1 x 1 torus


@pytest.mark.parametrize("flags", [C.DO_PERSISTENT, C.DO_PLAIN, GRAPH])
def test_random_seas_modes(flags):
    for seed, side in ((1, 64), (2, 97)):
        ref = check(W.wator_inputs(side, seed=seed), [1, 9, 30], flags=flags)
        assert ref.fish_born > 0 and ref.fish_eaten > 0 and ref.sharks_starved > 0


def test_per_type_capacity_and_empty_and_full_seas():
    ref = check(W.wator_inputs(80, seed=4), [5, 25], capacity=0)   # Fish 64 slots, Shark 32
    assert ref.sharks_born > 0
    check(W.wator_inputs(32, seed=6, fish24=0, shark24=0), [3])     # nothing at all
    check(W.wator_inputs(32, seed=7, fish24=1 << 24, shark24=0), [3])   # all fish: nobody moves
    check(W.wator_inputs(40, seed=8, fish24=0, shark24=1 << 23), [6])   # sharks only: all starve


def test_long_run_512():
    check(W.wator_inputs(512, seed=11), [100, 200], flags=GRAPH)


def test_full_config_2048_first_steps():
    # The benchmark sea (2048 x 2048, fish 0.30, sharks 0.05), its first 20
    # steps against the oracle (graph replay, as timed).
    check(W.wator_inputs(2048), [20], flags=GRAPH)


def test_benchmark_run_2048_200_steps_against_stored_oracle_digests():
    # The benchmark's run (2048 x 2048, fish 0.30, sharks 0.05, seed 24301,
    # graph replay) for all its 200 steps: the sea and the object churn at
    # every 50th step equal the oracle's (digests written by
    # tests/golden/make_golden.py), and no sticky flag is raised.
    import hashlib
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "wator_2048_200s_seed24301.json")))
    inp = W.wator_inputs(ref["side"], seed=ref["seed"])
    sea = apps.Wator(inp, RULES)
    sea.init()
    f0, s0 = ref["initial"]["fish"], ref["initial"]["sharks"]
    done = 0
    for cp in ref["checkpoints"]:
        sea.step(cp["step"] - done, GRAPH)
        done = cp["step"]
        got = sea.read()
        for f in ("kind", "age", "energy"):
            assert hashlib.sha256(np.ascontiguousarray(getattr(got, f)).tobytes()).hexdigest() == \
                cp[f"{f}_sha256"], f"{f} differs after {done} steps"
        st = got.stats
        assert st["allocs"] == [f0 + cp["fish_born"], s0 + cp["sharks_born"]]
        assert st["frees"] == [cp["fish_eaten"], cp["sharks_starved"]]
        assert st["live"] == [cp["fish"], cp["sharks"]]
    assert sea.heap.check() == {}
    sea.close()
