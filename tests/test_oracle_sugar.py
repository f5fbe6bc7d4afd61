"""Pins of the oracle's Sugarscape-style rules: hand-worked one- and two-agent
cases on a 5 x 5 torus, and invariants that hold at any size."""
import numpy as np
import pytest

from synth import rng
from synth import workloads as W

RULES = dict(W.SUGAR_RULES)
SEED = 77


def empty_state(orc, side=5):
    n = side * side
    z = lambda: np.zeros(n, dtype=np.int32)
    return orc.SugarState(side, z(), z(), np.zeros(n, dtype=np.uint8), z(), z(), z(), z())


def put(s, cell, sugar, metab, vision, age):
    s.occ[cell] = 1
    s.a_sugar[cell], s.a_metab[cell], s.a_vision[cell], s.a_age[cell] = sugar, metab, vision, age


def test_single_agent_moves_to_sugar_and_eats(orc):
    s = empty_state(orc)
    s.cap[13] = 3; s.sugar[13] = 3               # cell (3, 2)
    put(s, 12, sugar=5, metab=1, vision=1, age=0)  # cell (2, 2)
    r = orc.sugar_run(s, 1, SEED, RULES)
    assert list(np.nonzero(r.occ)[0]) == [13]
    assert (r.a_sugar[13], r.a_age[13]) == (5 + 3 - 1, 1)
    assert r.sugar[13] == 0 and r.moves == 1 and r.births == 0 and r.deaths == 0


def test_conflict_lowest_cell_index_wins(orc):
    s = empty_state(orc)
    s.cap[12] = 4; s.sugar[12] = 4
    put(s, 11, sugar=6, metab=2, vision=1, age=3)  # west of 12
    put(s, 13, sugar=6, metab=2, vision=1, age=3)  # east of 12
    r = orc.sugar_run(s, 1, SEED, RULES)
    assert sorted(np.nonzero(r.occ)[0]) == [12, 13]
    assert r.a_sugar[12] == 6 + 4 - 2            # the winner (from 11) ate
    assert r.a_sugar[13] == 6 - 2                # the loser stayed on an empty cell
    assert r.moves == 1


def test_stays_on_own_cell_when_tied(orc):
    s = empty_state(orc)
    s.cap[:] = 2; s.sugar[:] = 2
    put(s, 12, sugar=5, metab=1, vision=3, age=0)
    r = orc.sugar_run(s, 1, SEED, RULES)
    assert r.occ[12] == 1 and r.moves == 0 and r.a_sugar[12] == 6


def test_nearest_then_lowest_index_breaks_ties(orc):
    s = empty_state(orc, side=9)
    c = 4 * 9 + 4                                # centre (4, 4)
    for q in (c + 2, c - 2, c + 18):             # (6,4), (2,4), (4,6): distance 2
        s.cap[q] = 3; s.sugar[q] = 3
    put(s, c, sugar=5, metab=1, vision=4, age=0)
    r = orc.sugar_run(s, 1, SEED, RULES)
    assert r.occ[c - 2] == 1                     # equal sugar and distance: lowest index


def test_birth_rule_and_child_traits(orc):
    s = empty_state(orc)
    put(s, 12, sugar=30, metab=1, vision=1, age=20)
    r = orc.sugar_run(s, 1, SEED, RULES, step0=4)
    # No sugar anywhere: the agent stays, has 29 sugar at age 21 and is
    # fertile; its lowest-index empty neighbour is cell 7 (north of 12).
    assert sorted(np.nonzero(r.occ)[0]) == [7, 12]
    assert r.a_sugar[12] == 29 - 14 and r.a_sugar[7] == 14 and r.a_age[7] == 0
    hm = rng.hash4(SEED, rng.S_SUGAR_CHILD_METAB, 4, 7)
    hv = rng.hash4(SEED, rng.S_SUGAR_CHILD_VISION, 4, 7)
    assert r.a_metab[7] == int(rng.uniform_int(hm, 1, 4))
    assert r.a_vision[7] == int(rng.uniform_int(hv, 1, 6))
    assert r.births == 1


@pytest.mark.parametrize("age,sugar,dies", [(RULES["max_age"] - 1, 50, True),
                                            (RULES["max_age"] - 2, 50, False),
                                            (5, 1, True), (5, 2, False)])
def test_death_rules(orc, age, sugar, dies):
    s = empty_state(orc)
    put(s, 12, sugar=sugar, metab=1, vision=1, age=age)
    r = orc.sugar_run(s, 1, SEED, dict(RULES, repro_min=10 ** 6))
    assert (r.occ.sum() == 0) == dies and r.deaths == int(dies)


def test_invariants_random_medium(orc):
    inp = W.sugar_inputs(64, 900, seed=5)
    s = orc.SugarState(64, inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab,
                       inp.a_vision, inp.a_age)
    pop = int(s.occ.sum())
    for k in range(30):
        r = orc.sugar_run(s, 1, 5, RULES, step0=k)
        assert ((r.sugar >= 0) & (r.sugar <= r.cap)).all()
        m = r.occ.astype(bool)
        assert (r.a_sugar[m] > 0).all() and (r.a_age[m] < RULES["max_age"]).all()
        assert ((r.a_metab[m] >= 1) & (r.a_metab[m] <= 4)).all()
        assert ((r.a_vision[m] >= 1) & (r.a_vision[m] <= 6)).all()
        pop = pop + (r.births - s.births) - (r.deaths - s.deaths)
        assert int(r.occ.sum()) == pop
        s = r


def test_split_runs_equal_one_run(orc):
    inp = W.sugar_inputs(32, 200, seed=9)
    s = orc.SugarState(32, inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab,
                       inp.a_vision, inp.a_age)
    a = orc.sugar_run(s, 20, 9, RULES)
    b = orc.sugar_run(orc.sugar_run(s, 7, 9, RULES), 13, 9, RULES, step0=7)
    for f in ("sugar", "occ", "a_sugar", "a_metab", "a_vision", "a_age"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert (a.births, a.deaths, a.moves) == (b.births, b.deaths, b.moves)


def ledger(s):
    m = s.occ.astype(bool)
    return int(s.a_sugar[m].sum()) + int(s.sugar.sum())


@pytest.mark.parametrize("side,agents,seed,rules", [
    (64, 60, 5, RULES),                                             # births and deaths
    (48, 600, 6, dict(RULES, max_age=10 ** 6, fertile_min=2, fertile_max=1)),  # neither: every step checked
])
def test_sugar_ledger(orc, side, agents, seed, rules):
    # The sugar of all agents and all cells changes in a step by the regrowth
    # (each cell's sugar + 1, capped, minus its sugar), minus the metabolism of
    # the agents that started the step, minus the sugar the dead take with
    # them; eating moves sugar from a cell to an agent and a birth from the
    # parent to the child, so neither changes the total.  On steps without
    # deaths the last term is 0, and the equation is closed from the state
    # before the step alone.
    inp = W.sugar_inputs(side, agents, seed=seed)
    a_sugar = inp.a_sugar.copy()
    if rules is not RULES:
        a_sugar[inp.occ.astype(bool)] += 200  # no starvation within the run
    s = orc.SugarState(side, inp.sugar, inp.cap, inp.occ, a_sugar, inp.a_metab, inp.a_vision, inp.a_age)
    checked = births_checked = 0
    for k in range(40):
        r = orc.sugar_run(s, 1, seed, rules, step0=k)
        if r.deaths == s.deaths:
            regrow = int((np.minimum(s.sugar + 1, s.cap) - s.sugar).sum())
            metab = int(s.a_metab[s.occ.astype(bool)].sum())
            assert ledger(r) == ledger(s) + regrow - metab, k
            checked += 1
            births_checked += r.births - s.births
        s = r
    assert checked >= (40 if rules is not RULES else 5)
    if rules is RULES:
        assert births_checked > 0  # the parent-to-child transfer is among the checked steps
    if rules is not RULES:
        assert s.births == 0 and s.deaths == 0
