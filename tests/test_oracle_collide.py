"""Merging-bodies particle system oracle: hand-worked cases of attraction,
straight-line motion, merging (mass, momentum, centre of mass) and the
root/target rule, plus invariants (exact total mass, body count)."""
import numpy as np

import oracle
from synth import workloads as W


def state(*bodies):
    a = np.array(bodies, dtype=np.float32)
    return oracle.CollideState(a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy(), a[:, 3].copy(), a[:, 4].copy())


def test_lone_body_moves_in_a_straight_line():
    s = oracle.collide_run(state((1.0, 2.0, 1.0, -0.5, 3.0)), 8, dict(dt=0.25, eps2=0.01, r2_merge=0.0))
    assert (s.x[0], s.y[0], s.vx[0], s.vy[0], s.m[0]) == (3.0, 1.0, 1.0, -0.5, 3.0)


def test_two_bodies_attract_exactly():
    # unit masses 0.75 apart with softening 0.4375: r2 = 0.5625 + 0.4375 = 1, so
    # each accelerates by 0.75 towards the other (the self term adds exactly 0)
    s = oracle.collide_run(state((0.0, 0.0, 0.0, 0.0, 1.0), (0.75, 0.0, 0.0, 0.0, 1.0)), 1,
                           dict(dt=0.5, eps2=0.4375, r2_merge=0.0))
    assert (s.vx[0], s.vx[1]) == (0.375, -0.375)
    assert (s.x[0], s.x[1]) == (0.1875, 0.5625)


def test_symmetric_pair_stays_symmetric():
    s = oracle.collide_run(state((-0.3, 0.1, 0.0, 0.0, 2.0), (0.3, -0.1, 0.0, 0.0, 2.0)), 20,
                           dict(dt=0.01, eps2=0.01, r2_merge=0.0))
    assert s.x[0] == -s.x[1] and s.y[0] == -s.y[1] and s.vx[0] == -s.vx[1]


def test_merge_keeps_mass_momentum_and_centre():
    s = oracle.collide_run(state((0.0, 0.0, 1.0, 0.0, 1.0), (0.25, 0.0, -1.0, 0.0, 1.0)), 1,
                           dict(dt=0.0, eps2=1.0, r2_merge=0.25))
    assert s.merges == 1 and s.m[1] == 0.0
    assert (s.m[0], s.vx[0], s.x[0], s.y[0]) == (2.0, 0.0, 0.125, 0.0)


def test_roots_and_targets_along_a_chain():
    # 0 -- 1 -- 2 spaced 0.25 with merge radius 0.3: 0 is the only root, 1 merges
    # into it, 2 has no root in reach (0 is 0.5 away) and survives.
    s = oracle.collide_run(state((0.0, 0.0, 0.0, 0.0, 1.0), (0.25, 0.0, 0.0, 0.0, 1.0),
                                 (0.5, 0.0, 0.0, 0.0, 1.0)), 1, dict(dt=0.0, eps2=1.0, r2_merge=0.09))
    assert s.merges == 1 and list(s.m) == [2.0, 0.0, 1.0]
    assert s.x[0] == 0.125 and s.x[2] == 0.5


def test_random_mass_exact_and_count():
    inp = W.collide_inputs(300, seed=4, box=2.0)
    s0 = oracle.CollideState(inp.x, inp.y, inp.vx, inp.vy, inp.m)
    s = oracle.collide_run(s0, 15, W.COLLIDE_PARAMS)
    assert s.m.sum(dtype=np.float64) == inp.m.sum(dtype=np.float64)   # integer masses add exactly
    assert int((s.m > 0).sum()) == 300 - s.merges and s.merges > 0
    assert np.isfinite(s.x).all() and np.isfinite(s.vx).all()


def test_split_runs_equal_one_run():
    inp = W.collide_inputs(120, seed=2, box=2.0)
    s0 = oracle.CollideState(inp.x, inp.y, inp.vx, inp.vy, inp.m)
    a = oracle.collide_run(s0, 10, W.COLLIDE_PARAMS)
    b = oracle.collide_run(oracle.collide_run(s0, 4, W.COLLIDE_PARAMS), 6, W.COLLIDE_PARAMS)
    for f in ("x", "y", "vx", "vy", "m"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert a.merges == b.merges


def test_zero_merge_radius_never_merges():
    # The same dense bodies merge with the default radius and never with 0.
    inp = W.collide_inputs(512, seed=7, box=1.0)
    st = oracle.CollideState(inp.x, inp.y, inp.vx, inp.vy, inp.m)
    merged = oracle.collide_run(st, 3, W.COLLIDE_PARAMS)
    assert merged.merges > 0
    kept = oracle.collide_run(st, 3, dict(W.COLLIDE_PARAMS, r2_merge=0.0))
    assert kept.merges == 0
    assert np.array_equal(kept.m, inp.m)
