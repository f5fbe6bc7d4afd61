"""Device hierarchical bitmap (Sec. 2.1 operations, Sec. 3 / Alg. 2) against
the paper's cascade example, exact outcomes of concurrent storms, and
container consistency at quiescence."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd.heap import DeviceBitmap  # noqa: E402


WIDTHS = [64, 32]


def words_np(bm):
    return [w.cpu().numpy().view(np.uint64 if bm.width == 64 else np.uint32) for w in bm.level_words()]


def assert_consistent(bm):
    lv = words_np(bm)
    n, cw = bm.nbits, bm.width
    for l, w in enumerate(lv):
        # no bits at or beyond the level's size
        for i, x in enumerate(w):
            lo = cw * i
            if n - lo < cw:
                assert int(x) >> max(n - lo, 0) == 0, (l, i)
        if l + 1 < len(lv):
            up = lv[l + 1]
            for i, x in enumerate(w):
                assert ((int(up[i // cw]) >> (i % cw)) & 1) == (1 if int(x) else 0), (l, i)
        n = len(w)


def assert_equals_oracle(bm, ref):
    # Every level, container by container, equals the sequential model's.
    lv = words_np(bm)
    assert len(lv) == ref.nlevels
    for l, w in enumerate(lv):
        assert [int(x) for x in w] == [int(x) for x in ref.words(l)], l


def ops_tensor(kinds, poss):
    return torch.tensor(np.stack([kinds, poss], axis=1).astype(np.int32), device="cuda")


def test_width64_cascade_analogue_of_paper_example():
    # The paper's example (N = 32, 4-bit containers) at the real width: with
    # 64^3 bits, clearing the only set bit of container 1152 empties it, which
    # clears level-1 bit 1152 (emptying level-1 container 18), which clears
    # top bit 18.  Bit 3 keeps the branch of top bit 0 alive.
    bm = DeviceBitmap(64 ** 3)
    p1 = 18 * 4096
    r = bm.run(ops_tensor([C.BM_TRY_SET, C.BM_TRY_SET], [p1, 3]))
    assert r.tolist() == [1, 1]
    lv = words_np(bm)
    assert int(lv[2][0]) == (1 << 18) | 1
    r = bm.run(ops_tensor([C.BM_CLEAR], [p1]))
    assert r.tolist() == [0]
    lv = words_np(bm)
    assert int(lv[0][1152]) == 0 and int(lv[1][18]) == 0 and int(lv[2][0]) == 1
    assert_consistent(bm)


def test_width32_cascade_analogue_of_paper_example():
    # The same cascade with 32-bit containers (32^3 bits, three levels):
    # clearing the only set bit of level-0 container 576 = 18 * 32 clears
    # level-1 bit 576, which empties level-1 container 18 and clears top bit
    # 18.  Bit 3 keeps top bit 0.
    bm = DeviceBitmap(32 ** 3, width=32)
    p1 = 18 * 1024
    assert bm.run(ops_tensor([C.BM_TRY_SET, C.BM_TRY_SET], [p1, 3])).tolist() == [1, 1]
    lv = words_np(bm)
    assert len(lv) == 3 and int(lv[2][0]) == (1 << 18) | 1
    assert bm.run(ops_tensor([C.BM_CLEAR], [p1])).tolist() == [0]
    lv = words_np(bm)
    assert int(lv[0][576]) == 0 and int(lv[1][18]) == 0 and int(lv[2][0]) == 1
    assert_consistent(bm)


@pytest.mark.parametrize("width", WIDTHS)
@pytest.mark.parametrize("nbits,seed", [(4096, 1), (5000, 2), (64 ** 3 + 17, 3)])
def test_concurrent_try_ops_exact(nbits, seed, width):
    import oracle
    rng = np.random.default_rng(seed)
    init = rng.random(nbits) < 0.3
    bm = DeviceBitmap(nbits, width=width)
    pos0 = np.nonzero(init)[0]
    assert (bm.run(ops_tensor(np.full(len(pos0), C.BM_TRY_SET), pos0)).cpu().numpy() == 1).all()
    assert_consistent(bm)
    # One op per position, all concurrent: many wavefronts hit the same
    # containers, so cascades race with sets in the same container.
    n = min(nbits, 20000)
    pos = rng.permutation(nbits)[:n]
    kinds = rng.integers(0, 2, size=n)  # 0 try_set, 1 try_clear
    res = bm.run(ops_tensor(kinds, pos)).cpu().numpy()
    exp_res = np.where(kinds == 0, ~init[pos], init[pos]).astype(np.int32)
    assert np.array_equal(res, exp_res)
    final = init.copy()
    final[pos[kinds == 0]] = True
    final[pos[kinds == 1]] = False
    lv0 = words_np(bm)[0]
    got = np.unpackbits(lv0.view(np.uint8), bitorder="little")[:nbits].astype(bool)
    assert np.array_equal(got, final)
    assert_consistent(bm)
    ref = oracle.Bitmap(nbits, width)
    for p_ in np.nonzero(final)[0]:
        ref.try_set(int(p_))
    assert_equals_oracle(bm, ref)


@pytest.mark.parametrize("width", WIDTHS)
@pytest.mark.parametrize("nbits", [1, 32, 33, 64, 65, 4097, 30000])
def test_find_clear_drains_exactly(nbits, width):
    bm = DeviceBitmap(nbits, all_set=True, width=width)
    assert_consistent(bm)
    n = nbits + 100
    rng = np.random.default_rng(nbits)
    starts = torch.tensor(rng.integers(0, 2 ** 31, size=n).astype(np.int32), device="cuda")
    res = bm.run(ops_tensor(np.full(n, C.BM_FIND_CLEAR), np.zeros(n, np.int64)), starts).cpu().numpy()
    got = res[res >= 0]
    assert len(got) == nbits and len(set(got.tolist())) == nbits     # each bit handed out once
    assert (res[res < 0] == -1).sum() == 100
    assert all(int(w.abs().sum()) == 0 for w in bm.level_words())


@pytest.mark.parametrize("width", WIDTHS)
def test_try_find_set_at_quiescence_brute_force(width):
    rng = np.random.default_rng(5)
    for nbits, density in [(300, 0.0), (300, 0.01), (4096, 0.001), (70000, 0.0001)]:
        bm = DeviceBitmap(nbits, width=width)
        init = rng.random(nbits) < density
        pos0 = np.nonzero(init)[0]
        if len(pos0):
            bm.run(ops_tensor(np.full(len(pos0), C.BM_TRY_SET), pos0))
        n = 256
        starts = torch.tensor(rng.integers(0, 2 ** 31, size=n).astype(np.int32), device="cuda")
        res = bm.run(ops_tensor(np.full(n, C.BM_TRY_FIND_SET), np.zeros(n, np.int64)), starts).cpu().numpy()
        if len(pos0) == 0:
            assert (res == -1).all()
        else:
            assert np.isin(res, pos0).all()


@pytest.mark.parametrize("width", WIDTHS)
def test_set_clear_pairs_meet(width):
    # set(pos) and clear(pos) issued together on a clear bit: clear retries
    # until the set lands (Sec. 2.1), so both finish and the bit ends clear.
    nbits = 8192
    bm = DeviceBitmap(nbits, width=width)
    pos = np.arange(0, nbits, 8)
    kinds = np.concatenate([np.full(len(pos), C.BM_CLEAR), np.full(len(pos), C.BM_SET)])
    res = bm.run(ops_tensor(kinds, np.concatenate([pos, pos]))).cpu().numpy()
    assert (res == 0).all()
    assert all(int(w.abs().sum()) == 0 for w in bm.level_words())


def inject(bm, edits):
    """Host-side edits of raw level words (a summary left behind by an update
    still on its way): edits = [(level, container, bits to OR, bits to clear)]."""
    lv = bm.level_words()
    for level, c, set_bits, clear_bits in edits:
        w = lv[level][c:c + 1]
        dt = np.uint64 if bm.width == 64 else np.uint32
        x = (int(w.cpu().numpy().view(dt)[0]) | set_bits) & ~clear_bits & ((1 << bm.width) - 1)
        w.copy_(torch.from_numpy(np.array([x], dtype=dt).view(np.int64 if bm.width == 64 else np.int32)))


@pytest.mark.parametrize("width", WIDTHS)
def test_stale_set_summaries_never_yield_a_clear_bit(width):
    # Summary bits left set above empty containers (as while a clear's
    # cascade is on its way): searches that descend into them must fail or
    # retry elsewhere, never return a clear bit; a drain still hands out
    # every real bit exactly once and leaves level 0 empty.
    nbits = 64 ** 3
    rng = np.random.default_rng(21)
    bm = DeviceBitmap(nbits, width=width)
    real = np.sort(rng.choice(nbits, 300, replace=False))
    assert (bm.run(ops_tensor(np.full(len(real), C.BM_TRY_SET), real)).cpu().numpy() == 1).all()
    used = set((real // width).tolist())
    empty = [c for c in rng.permutation(nbits // width)[:400].tolist() if c not in used][:200]
    edits = []
    for c in empty:
        # The level-1 bit of empty container c, and the bits above it, so
        # that searches do reach it.
        pos, level = c, 1
        while level < len(bm.level_words()):
            edits.append((level, pos // width, 1 << (pos % width), 0))
            pos //= width
            level += 1
    inject(bm, edits)
    n = 4096
    starts = torch.tensor(rng.integers(0, 2 ** 31, size=n).astype(np.int32), device="cuda")
    res = bm.run(ops_tensor(np.full(n, C.BM_TRY_FIND_SET), np.zeros(n, np.int64)), starts).cpu().numpy()
    assert np.isin(res[res >= 0], real).all()
    assert (res >= 0).any()
    m = len(real)
    starts = torch.tensor(rng.integers(0, 2 ** 31, size=m).astype(np.int32), device="cuda")
    got = bm.run(ops_tensor(np.full(m, C.BM_FIND_CLEAR), np.zeros(m, np.int64)), starts).cpu().numpy()
    assert sorted(got.tolist()) == real.tolist()
    assert int(bm.level_words()[0].abs().sum()) == 0


@pytest.mark.parametrize("width", WIDTHS)
def test_stale_clear_summaries_hide_bits_until_the_cascade_lands(width):
    # Set bits whose summary bit is still clear (as while a set's cascade is
    # on its way): a search cannot reach them, so find_clear reports FAIL
    # although bits are set (a FAIL does not prove the bitmap empty); once the
    # host completes the cascade, a drain returns exactly those bits.
    nbits = 64 ** 3
    bm = DeviceBitmap(nbits, width=width)
    real = np.array([5 * width + 1, 5 * width + 7, 900 * width + 3])
    assert (bm.run(ops_tensor(np.full(len(real), C.BM_TRY_SET), real)).cpu().numpy() == 1).all()
    before = [w.clone() for w in bm.level_words()]
    lv = bm.level_words()
    for lvl in range(1, len(lv)):
        lv[lvl].zero_()  # every summary bit clear: only level 0 holds the bits
    n = 64
    starts = torch.tensor(np.arange(n, dtype=np.int32) * 7919, device="cuda")
    res = bm.run(ops_tensor(np.full(n, C.BM_TRY_FIND_SET), np.zeros(n, np.int64)), starts).cpu().numpy()
    assert (res == -1).all()
    res = bm.run(ops_tensor(np.full(4, C.BM_FIND_CLEAR), np.zeros(4, np.int64)), starts[:4]).cpu().numpy()
    assert (res == -1).all()
    assert np.array_equal(words_np(bm)[0], before[0].cpu().numpy().view(words_np(bm)[0].dtype))
    for lvl in range(1, len(lv)):
        lv[lvl].copy_(before[lvl])  # the cascades land
    assert_consistent(bm)
    got = bm.run(ops_tensor(np.full(len(real), C.BM_FIND_CLEAR), np.zeros(len(real), np.int64)),
                 starts[:len(real)]).cpu().numpy()
    assert sorted(got.tolist()) == real.tolist()
    assert all(int(w.abs().sum()) == 0 for w in bm.level_words())
