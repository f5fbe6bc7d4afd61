"""Wa-Tor oracle (fish and sharks, Dewdney's rules in the synchronous reading
the oracle's header states) against hand-worked cases and invariants that
hold at any size: a lone fish wanders and breeds, a boxed-in fish neither
moves nor breeds, the lowest requesting cell wins a contested cell, a shark
eats a neighbouring fish and starves without one, and populations change
exactly by the counted births, meals and starvations."""
import numpy as np

import oracle
from synth import workloads as W

RULES = dict(fish_breed=3, shark_breed=10, starve=3)


def grid(side, cells):
    """cells: {(x, y): (kind, age, energy)}"""
    k = np.zeros((side, side), np.int32)
    a = np.zeros((side, side), np.int32)
    e = np.zeros((side, side), np.int32)
    for (x, y), (kk, aa, ee) in cells.items():
        k[y, x], a[y, x], e[y, x] = kk, aa, ee
    return oracle.WatorState(k, a, e)


def neighbours(side, x, y):
    return {((x + dx) % side, (y + dy) % side) for dx, dy in ((0, -1), (1, 0), (0, 1), (-1, 0))}


def test_lone_fish_moves_to_a_neighbour_and_breeds_on_schedule():
    s = grid(7, {(3, 3): (1, 0, 0)})
    pos = (3, 3)
    for t in range(6):
        s = oracle.wator_run(s, 1, 5, RULES, step0=t)
        fish = {(int(x), int(y)) for y, x in zip(*np.nonzero(s.kind == 1))}
        if t == 2:  # third move: age reaches fish_breed, a newborn stays behind
            assert len(fish) == 2 and pos in fish
            assert s.fish_born == 1
            new = (fish - {pos}).pop()
            assert new in neighbours(7, *pos)
            assert s.age[pos[1], pos[0]] == 0 and s.age[new[1], new[0]] == 0
            break
        assert len(fish) == 1
        new = fish.pop()
        assert new in neighbours(7, *pos)
        assert s.age[new[1], new[0]] == t + 1
        pos = new


def test_boxed_in_fish_neither_moves_nor_breeds():
    # A full 2 x 2 torus of fish: nobody has an empty neighbour.
    s = grid(2, {(x, y): (1, 5, 0) for x in range(2) for y in range(2)})
    s = oracle.wator_run(s, 4, 1, RULES)
    assert (s.kind == 1).all() and (s.age == 9).all() and s.fish_born == 0


def test_lowest_requesting_cell_wins_the_only_free_cell():
    # 3 x 3 torus full of fish but the centre: cells 1, 3, 5 and 7 each have
    # the centre as their only empty neighbour, so each must request it; the
    # corners have none.  Cell 1 (x=1, y=0) wins.
    cells = {(x, y): (1, 0, 0) for x in range(3) for y in range(3) if (x, y) != (1, 1)}
    s = oracle.wator_run(grid(3, cells), 1, 9, RULES)
    assert s.kind[1, 1] == 1 and s.age[1, 1] == 1      # the mover, one step older
    assert s.kind[0, 1] == 0                            # cell 1 left empty (age 1 < 3)
    assert (s.kind == 1).sum() == 8
    for (x, y) in [(0, 1), (2, 1), (1, 2), (0, 0), (2, 0), (0, 2), (2, 2)]:
        assert s.kind[y, x] == 1 and s.age[y, x] == 1
    # With age 2 the winner breeds: the centre and cell 1 both hold fish, age 0.
    cells = {(x, y): (1, 2, 0) for x in range(3) for y in range(3) if (x, y) != (1, 1)}
    s = oracle.wator_run(grid(3, cells), 1, 9, RULES)
    assert (s.kind == 1).all() and s.age[1, 1] == 0 and s.age[0, 1] == 0 and s.fish_born == 1


def test_shark_eats_a_neighbouring_fish():
    # 2 x 2 torus: a shark at cell 0 and fish elsewhere; no fish can move
    # (no empty cell), the shark's neighbours are the fish at 1 and 2.
    s = grid(2, {(0, 0): (2, 0, 1), (1, 0): (1, 0, 0), (0, 1): (1, 0, 0), (1, 1): (1, 0, 0)})
    s = oracle.wator_run(s, 1, 3, RULES)
    assert s.fish_eaten == 1 and s.sharks_starved == 0
    assert s.kind[0, 0] == 0                              # moved away, too young to breed
    assert sorted([int(s.kind[0, 1]), int(s.kind[1, 0])]) == [1, 2]
    y, x = np.argwhere(s.kind == 2)[0]
    assert s.energy[y, x] == RULES["starve"] and s.age[y, x] == 1
    assert s.kind[1, 1] == 1


def test_shark_without_fish_starves_on_schedule():
    s = grid(5, {(2, 2): (2, 0, 3)})
    for t in range(2):
        s = oracle.wator_run(s, 1, 4, RULES, step0=t)
        assert (s.kind == 2).sum() == 1
        y, x = np.argwhere(s.kind == 2)[0]
        assert s.energy[y, x] == 3 - (t + 1)
    s = oracle.wator_run(s, 1, 4, RULES, step0=2)   # energy 1: no move, then 0: dies
    assert (s.kind == 2).sum() == 0 and s.sharks_starved == 1


def test_populations_change_exactly_by_the_counts_random():
    for seed in (1, 2):
        inp = W.wator_inputs(64, seed=seed)
        s0 = oracle.WatorState(inp.kind, inp.age, inp.energy)
        s = oracle.wator_run(s0, 60, seed, W.WATOR_RULES)
        f0, k0 = int((inp.kind == 1).sum()), int((inp.kind == 2).sum())
        assert int((s.kind == 1).sum()) == f0 + s.fish_born - s.fish_eaten
        assert int((s.kind == 2).sum()) == k0 + s.sharks_born - s.sharks_starved
        sharks = s.kind == 2
        assert (s.energy[sharks] >= 1).all() and (s.energy[sharks] <= W.WATOR_RULES["starve"]).all()
        assert s.fish_born > 0 and s.fish_eaten > 0 and s.sharks_born > 0 and s.sharks_starved > 0


def test_split_runs_equal_one_run_and_zero_steps():
    inp = W.wator_inputs(48, seed=3)
    s0 = oracle.WatorState(inp.kind, inp.age, inp.energy)
    one = oracle.wator_run(s0, 25, 3, W.WATOR_RULES)
    a = oracle.wator_run(s0, 10, 3, W.WATOR_RULES)
    b = oracle.wator_run(a, 15, 3, W.WATOR_RULES, step0=10)
    for f in ("kind", "age", "energy"):
        assert np.array_equal(getattr(one, f), getattr(b, f))
    assert (one.fish_born, one.fish_eaten) == (b.fish_born, b.fish_eaten)
    z = oracle.wator_run(s0, 0, 3, W.WATOR_RULES)
    assert np.array_equal(z.kind, inp.kind)
