"""Merging bodies (collisions) on the device against the oracle: bit-exact
positions, velocities and masses by id (every float operation is rounded
once, in the oracle's order), and exact object churn (bodies deleted =
merges)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd import apps  # noqa: E402
from synth import workloads as W  # noqa: E402

GRAPH = C.DO_PERSISTENT | C.GRAPH
FIELDS = ("x", "y", "vx", "vy", "m")


def check(inp, params, split, flags=C.DO_PERSISTENT):
    sim = apps.Collisions(inp, params)
    sim.init()
    ref = oracle.CollideState(inp.x, inp.y, inp.vx, inp.vy, inp.m)
    done = 0
    for k in split:
        sim.step(k, flags)
        ref = oracle.collide_run(ref, k, params)
        done += k
        got = sim.read()
        for f in FIELDS:
            assert np.array_equal(getattr(got, f).view(np.uint32), getattr(ref, f).view(np.uint32)), \
                f"{f} differs after {done} steps"
    st = got.stats
    assert st["frees"] == [ref.merges]
    assert st["live"] == [int((ref.m > 0).sum())]
    assert sim.heap.check() == {}
    return ref


def inputs_of(*bodies):
    a = np.array(bodies, dtype=np.float32)
    return W.CollideInputs(len(a), 1, *[a[:, k].copy() for k in range(5)])


def test_hand_cases():
    # attraction with exact values, a merge, and a chain (see the oracle tests)
    check(inputs_of((0.0, 0.0, 0.0, 0.0, 1.0), (0.75, 0.0, 0.0, 0.0, 1.0)), dict(dt=0.5, eps2=0.4375, r2_merge=0.0),
          [1, 1])
    check(inputs_of((0.0, 0.0, 1.0, 0.0, 1.0), (0.25, 0.0, -1.0, 0.0, 1.0)), dict(dt=0.0, eps2=1.0, r2_merge=0.25),
          [1])
    r = check(inputs_of((0.0, 0.0, 0.0, 0.0, 1.0), (0.25, 0.0, 0.0, 0.0, 1.0), (0.5, 0.0, 0.0, 0.0, 1.0)),
              dict(dt=0.0, eps2=1.0, r2_merge=0.09), [1])
    assert r.merges == 1


@pytest.mark.parametrize("flags", [C.DO_PERSISTENT, C.DO_PLAIN, GRAPH])
def test_random_bodies_modes(flags):
    inp = W.collide_inputs(700, seed=3, box=2.0)
    r = check(inp, W.COLLIDE_PARAMS, [1, 5, 14], flags=flags)
    assert r.merges > 0


def test_bodies_absent_at_start_and_per_type_capacity():
    inp = W.collide_inputs(300, seed=5, box=1.5)
    inp.m[::7] = 0.0  # ids with no body
    sim = apps.Collisions(inp, W.COLLIDE_PARAMS, capacity=32)
    sim.init()
    sim.step(10, GRAPH)
    ref = oracle.collide_run(oracle.CollideState(inp.x, inp.y, inp.vx, inp.vy, inp.m), 10, W.COLLIDE_PARAMS)
    got = sim.read()
    for f in FIELDS:
        assert np.array_equal(getattr(got, f).view(np.uint32), getattr(ref, f).view(np.uint32))


def test_full_config_4096_bodies_50_steps():
    # 4096 bodies in an 8 x 8 box, masses U{1..4}/1024, dt 0.01, eps2 0.01,
    # merge radius 0.01, 50 steps (graph replay).
    inp = W.collide_inputs(4096)
    r = check(inp, W.COLLIDE_PARAMS, [25, 25], flags=GRAPH)
    assert r.merges > 100


def test_nbody_mode_no_merge_radius():
    # Merge radius 0: no body ever merges (the nbody application); a step is
    # the force and move do-alls only.  Dense bodies that would merge with a
    # positive radius.
    inp = W.collide_inputs(2048, seed=7, box=2.0)
    params = dict(W.COLLIDE_PARAMS, r2_merge=0.0)
    ref = check(inp, params, [7, 13])
    assert ref.merges == 0
    assert int((ref.m > 0).sum()) == 2048


def test_benchmark_size_first_step():
    # The benchmark's 65,536 bodies in a 32 x 32 box, its first step (graph
    # replay, as timed) against the oracle, bit for bit.
    inp = W.collide_inputs(65536, box=32.0)
    ref = check(inp, W.COLLIDE_PARAMS, [1], flags=GRAPH)
    assert ref.merges > 0


@pytest.mark.parametrize("name,merge", [("collisions", True), ("nbody", False)])
def test_benchmark_run_against_stored_oracle_digests(name, merge):
    # The benchmark's 65,536 bodies in a 32 x 32 box for all its 20 steps
    # (graph replay, as timed): every body's position, velocity and mass,
    # bit for bit, at every fifth step equal the oracle's (digests written by
    # tests/golden/make_golden.py), and the merges and live bodies too.
    import hashlib
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      f"{name}_65536_20s_seed24301.json")))
    params = W.COLLIDE_PARAMS if merge else dict(W.COLLIDE_PARAMS, r2_merge=0.0)
    inp = W.collide_inputs(ref["bodies"], seed=ref["seed"], box=32.0)
    sim = apps.Collisions(inp, params)
    sim.init()
    done = 0
    for cp in ref["checkpoints"]:
        sim.step(cp["step"] - done, GRAPH)
        done = cp["step"]
        got = sim.read()
        for f in FIELDS:
            h = hashlib.sha256(np.ascontiguousarray(getattr(got, f).view(np.uint32)).tobytes()).hexdigest()
            assert h == cp[f + "_sha256"], f"{f} differs after {done} steps"
        assert got.stats["frees"] == [cp["merges"]] and got.stats["live"] == [cp["live"]]
    assert sim.heap.check() == {}
