"""Per-type block capacities (Sec. 2): the smallest type has 64 slots and
fixes the block size; other types get the largest power of two of their
objects that fits.  Pinned by worked cases of that rule."""
import oracle


def caps(sizes):
    return [oracle.type_capacity(sizes, t) for t in range(len(sizes))]


def test_single_and_equal_types_have_64():
    assert caps([12]) == [64]
    assert caps([8, 8, 8]) == [64, 64, 64]


def test_smallest_type_always_64_whatever_its_position():
    assert caps([16, 8]) == [32, 64]
    assert caps([8, 16]) == [64, 32]


def test_powers_of_two_floor():
    # 64 * 8 / 12 = 42.7 -> 32; 64 * 8 / 24 = 21.3 -> 16; 64 * 8 / 20 = 25.6 -> 16
    assert caps([8, 12, 24, 20]) == [64, 32, 16, 16]
    # exact fits stay exact
    assert caps([4, 8, 16, 32, 256]) == [64, 32, 16, 8, 1]


def test_huge_type_gets_one_slot():
    assert caps([4, 4 * 64]) == [64, 1]
    assert caps([4, 4 * 64 + 4]) == [64, 1]  # larger than a block: still one slot


def test_block_bytes_never_exceeded_below_the_single_slot_case():
    for sizes in ([4, 12, 28], [8, 36, 60, 124], [16, 20, 24, 28, 32, 40, 48, 64]):
        block = 64 * min(sizes)
        for t, s in enumerate(sizes):
            c = oracle.type_capacity(sizes, t)
            assert c & (c - 1) == 0 and 1 <= c <= 64
            assert c * s <= block or c == 1
            assert c == 64 or 2 * c * s > block   # the largest power of two that fits
