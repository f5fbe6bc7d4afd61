"""Pins of the oracle's Game of Life (B3/S23 on a torus): textbook patterns,
hand-counted candidate/birth/death numbers, and the glider's period on a
torus."""
import numpy as np
import pytest


def grid_with(w, h, cells):
    g = np.zeros((h, w), dtype=np.uint8)
    for x, y in cells:
        g[y % h, x % w] = 1
    return g


def test_empty_stays_empty(orc):
    g, c = orc.gol_run(np.zeros((9, 7), np.uint8), 5)
    assert g.sum() == 0 and c.sum() == 0


@pytest.mark.parametrize("cells", [
    [(1, 1), (2, 1), (1, 2), (2, 2)],                              # block
    [(2, 1), (3, 1), (1, 2), (4, 2), (2, 3), (3, 3)],              # beehive
    [(1, 1), (2, 1), (1, 2), (3, 2), (2, 3)],                      # boat
])
def test_still_lifes(orc, cells):
    g0 = grid_with(8, 8, cells)
    g, c = orc.gol_run(g0, 6)
    assert np.array_equal(g, g0)
    assert c[:, 1].sum() == 0 and c[:, 2].sum() == 0


def test_blinker_period_two_and_counts(orc):
    g0 = grid_with(5, 5, [(2, 1), (2, 2), (2, 3)])
    g1, c = orc.gol_step(g0)
    assert np.array_equal(g1, grid_with(5, 5, [(1, 2), (2, 2), (3, 2)]))
    # Hand count: the 3x5 neighbourhood of the vertical bar holds 15 cells,
    # 12 of them dead (candidates); two are born and the two tips die.
    assert list(c) == [12, 2, 2, 3]
    g2, _ = orc.gol_step(g1)
    assert np.array_equal(g2, g0)


def test_glider_translates_and_wraps(orc):
    glider = [(1, 0), (2, 1), (0, 2), (1, 2), (2, 2)]
    W = 10
    g0 = grid_with(W, W, glider)
    g4, _ = orc.gol_run(g0, 4)
    assert np.array_equal(g4, grid_with(W, W, [(x + 1, y + 1) for x, y in glider]))
    gw, c = orc.gol_run(g0, 4 * W)
    assert np.array_equal(gw, g0)
    assert (c[:, 3] == 5).all()                  # population is always 5


def test_rectangular_torus_wraps_both_axes(orc):
    # A blinker straddling the seam of a 6 x 5 torus behaves like any blinker.
    g0 = grid_with(6, 5, [(5, 0), (0, 0), (1, 0)])
    g2, _ = orc.gol_run(g0, 2)
    assert np.array_equal(g2, g0)
    g1, _ = orc.gol_step(g0)
    assert np.array_equal(g1, grid_with(6, 5, [(0, 4), (0, 0), (0, 1)]))


def test_full_grid_dies(orc):
    g, c = orc.gol_step(np.ones((6, 6), np.uint8))
    assert g.sum() == 0 and list(c) == [0, 0, 36, 0]


def test_counts_brute_force_small(orc):
    rng = np.random.default_rng(1)
    for _ in range(20):
        h, w = rng.integers(3, 12, size=2)
        g0 = (rng.random((h, w)) < 0.3).astype(np.uint8)
        g1, c = orc.gol_step(g0)
        cand = births = deaths = 0
        for y in range(h):
            for x in range(w):
                n = sum(g0[(y + dy) % h, (x + dx) % w] for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                        if (dx, dy) != (0, 0))
                if g0[y, x]:
                    deaths += n not in (2, 3)
                    assert g1[y, x] == (n in (2, 3))
                else:
                    cand += n > 0
                    births += n == 3
                    assert g1[y, x] == (n == 3)
        assert list(c) == [cand, births, deaths, int(g1.sum())]
