"""Nagel-Schreckenberg traffic oracle against hand-worked cases of the four
rules (accelerate, brake to the gap, dawdle, move; cars enter at the first
cell and leave past the last) and invariants that hold at any size."""
import numpy as np

import oracle
from synth import workloads as W

NO_RANDOM = dict(vmax=5, p_slow24=0, p_in24=0)


def road(length, cars):
    v = np.full((1, length), -1, np.int32)
    for i, s in cars.items():
        v[0, i] = s
    return v


def cars_of(v):
    return {int(i): int(v[0, i]) for i in np.nonzero(v[0] >= 0)[0]}


def test_free_flow_accelerates_to_vmax_and_leaves():
    v = road(30, {0: 0})
    pos = []
    for _ in range(7):
        r = oracle.traffic_run(v, 1, 1, NO_RANDOM)
        v = r.vel
        pos.append(cars_of(v))
    assert pos == [{1: 1}, {3: 2}, {6: 3}, {10: 4}, {15: 5}, {20: 5}, {25: 5}]
    r = oracle.traffic_run(v, 1, 1, NO_RANDOM)
    assert cars_of(r.vel) == {} and r.exits == 1 and r.entries == 0


def test_jam_dissolves_from_the_front():
    v = road(6, {i: 0 for i in range(6)})
    r1 = oracle.traffic_run(v, 1, 1, NO_RANDOM)       # only the front car moves: it leaves
    assert cars_of(r1.vel) == {i: 0 for i in range(5)} and r1.exits == 1
    r2 = oracle.traffic_run(r1.vel, 1, 1, NO_RANDOM)  # the new front car starts at speed 1
    assert cars_of(r2.vel) == {0: 0, 1: 0, 2: 0, 3: 0, 5: 1}
    r3 = oracle.traffic_run(r2.vel, 1, 1, NO_RANDOM)  # it leaves (5 + 2 >= 6); the next starts
    assert cars_of(r3.vel) == {0: 0, 1: 0, 2: 0, 4: 1} and r3.exits == 1


def test_brake_to_gap_then_follow():
    # A fast car behind a slow one stops right behind it.
    v = road(20, {2: 5, 5: 0})
    r = oracle.traffic_run(v, 1, 1, NO_RANDOM)
    assert cars_of(r.vel) == {4: 2, 6: 1}


def test_always_dawdling_car_never_moves():
    v = road(12, {3: 0})
    r = oracle.traffic_run(v, 10, 1, dict(vmax=5, p_slow24=1 << 24, p_in24=0))
    assert cars_of(r.vel) == {3: 0}


def test_entries_whenever_the_first_cell_is_free():
    v = road(50, {})
    r = oracle.traffic_run(v, 4, 1, dict(vmax=5, p_slow24=0, p_in24=1 << 24))
    # step 1: a enters at 0.  step 2: a -> 1 (speed 1); b enters at 0.
    # step 3: a -> 3 (speed 2); b sees a in cell 1: gap 0, stays; no entry.
    # step 4: a -> 6 (speed 3); b -> 1 (speed 1); c enters at 0.
    assert r.entries == 3 and r.exits == 0
    assert cars_of(r.vel) == {0: 0, 1: 1, 6: 3}


def test_conservation_and_speed_bounds_random():
    inp = W.traffic_inputs(40, 300, seed=7)
    v0 = inp.vel
    r = oracle.traffic_run(v0, 60, 7, W.TRAFFIC_RULES)
    assert int((r.vel >= 0).sum()) == int((v0 >= 0).sum()) + r.entries - r.exits
    assert r.vel.min() >= -1 and r.vel.max() <= W.TRAFFIC_RULES["vmax"]
    assert r.entries > 0 and r.exits > 0


def test_split_runs_equal_one_run_and_zero_steps():
    inp = W.traffic_inputs(8, 64, seed=3)
    a = oracle.traffic_run(inp.vel, 30, 3, W.TRAFFIC_RULES)
    b1 = oracle.traffic_run(inp.vel, 12, 3, W.TRAFFIC_RULES)
    b2 = oracle.traffic_run(b1.vel, 18, 3, W.TRAFFIC_RULES, step0=12)
    assert np.array_equal(a.vel, b2.vel)
    assert a.entries == b1.entries + b2.entries and a.exits == b1.exits + b2.exits
    z = oracle.traffic_run(inp.vel, 0, 3, W.TRAFFIC_RULES)
    assert np.array_equal(z.vel, inp.vel) and z.entries == z.exits == 0
