"""Pins of the oracle's hierarchical bitmap model (paper Sec. 2.1, Sec. 3, Alg. 2).

The model is checked against the paper's worked example (figure on clearing
a bit in a width-4 hierarchy), the operation contracts of Sec. 2.1, container
consistency, the nesting rule, and brute force on small bitmaps."""
import random

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")


def test_paper_example_width4_cascade(orc):
    # Sec. 3, figure "bitmap clear example": N = 32 bits with 4-bit containers.
    # clear(18) empties container 4, which clears bit 4 of the nested bitmap;
    # that empties nested container 1, which clears bit 1 one level up.
    b = orc.Bitmap(32, width=4)
    assert b.nlevels == 3                       # 32 -> 8 -> 2 bits
    assert [len(b.words(l)) for l in range(3)] == [8, 2, 1]
    assert b.set(18) and b.set(2)               # bit 2 keeps other containers busy
    assert int(b.words(1)[1]) == 0b0001         # nested bit 4 = container 1, bit 0
    assert int(b.words(2)[0]) == 0b11
    assert b.clear(18)
    assert b.trace() == [(0, 18), (1, 4), (2, 1)]
    assert int(b.words(2)[0]) == 0b01           # only the branch of bit 2 remains
    assert b.try_find_set() == 2


def test_try_clear_truth_table(orc):
    # Alg. 2: success iff the bit was set; the nested clear happens only when
    # the cleared bit was the container's last one.
    b = orc.Bitmap(256, width=64)
    assert not b.try_clear(5)                   # already clear: false, no cascade
    assert b.trace() == []
    b.set(5); b.set(6)
    assert b.try_clear(5)                       # not the last bit: no cascade
    assert b.trace() == [(0, 5)]
    assert int(b.words(1)[0]) == 1
    assert b.try_clear(6)                       # last bit: cascade to level 1
    assert b.trace() == [(0, 5), (0, 6), (1, 0)]
    assert int(b.words(1)[0]) == 0


def test_try_set_contract(orc):
    b = orc.Bitmap(130, width=64)
    assert b.try_set(129)
    assert not b.try_set(129)                   # already set: false
    assert int(b.words(1)[0]) == 0b100          # container 2 is non-empty
    assert b.get(129)


@pytest.mark.parametrize("n,levels", [(1, 1), (64, 1), (65, 2), (4096, 2), (4097, 3),
                                      (262144, 3), (262145, 4)])
def test_nesting_rule(orc, n, levels):
    # Sec. 3: a nested bitmap of ceil(N/64) bits exists iff N > 64.
    assert orc.Bitmap(n).nlevels == levels


@pytest.mark.parametrize("width", [4, 8, 64])
def test_random_ops_brute_force(orc, width):
    rnd = random.Random(7 + width)
    n = 300
    b = orc.Bitmap(n, width=width)
    model = set()
    for _ in range(4000):
        op = rnd.randrange(4)
        pos = rnd.randrange(n)
        if op == 0:
            assert b.try_set(pos) == (pos not in model)
            model.add(pos)
        elif op == 1:
            assert b.try_clear(pos) == (pos in model)
            model.discard(pos)
        elif op == 2:
            i = b.try_find_set()
            if model:
                assert i == min(model)           # the model picks the lowest set bit
            else:
                assert i == orc.FAIL
        else:
            i = b.find_clear()
            if model:
                assert i in model
                model.discard(i)
            else:
                assert i == orc.FAIL
        if rnd.random() < 0.05:
            # Container consistency: every nested bit is the OR of its container.
            for l in range(b.nlevels - 1):
                lower, upper = b.words(l), b.words(l + 1)
                for i, w in enumerate(lower):
                    assert ((int(upper[i // width]) >> (i % width)) & 1) == (1 if w else 0)
    got = {i for i in range(n) if b.get(i)}
    assert got == model


def test_full_bitmap_drains_in_order(orc):
    b = orc.Bitmap(5000, all_set=True)
    out = [b.find_clear() for _ in range(5000)]
    assert out == list(range(5000))
    assert b.find_clear() == orc.FAIL
    assert all(int(w) == 0 for l in range(b.nlevels) for w in b.words(l))


def test_all_set_bits_stop_at_size(orc):
    b = orc.Bitmap(70, all_set=True)
    w0 = b.words(0)
    assert int(w0[0]) == (1 << 64) - 1 and int(w0[1]) == (1 << 6) - 1
    assert int(b.words(1)[0]) == 0b11
