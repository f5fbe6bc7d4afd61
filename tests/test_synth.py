"""The shared input generators: pinned to the published SplitMix64 output and
to the distributions the workloads name."""
import os

import numpy as np

from synth import rng
from synth import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_vectors.txt")


def _vectors():
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            vals = [int(v) for v in line.split()]
            yield vals[0], vals[1:]


def test_mix64_matches_published_splitmix64():
    for seed, outs in _vectors():
        assert rng.splitmix64_sequence(seed, len(outs)) == outs


def test_oracle_mix64_matches_published_splitmix64(orc):
    for seed, outs in _vectors():
        state = seed
        for o in outs:
            state = (state + rng.GOLDEN) & rng.MASK64
            assert orc.mix64(state) == o


def test_hash_agrees_between_generator_and_oracle(orc):
    for a, b in [(0, 0), (1, 2), (2 ** 63, 5), (12345, 2 ** 40)]:
        assert int(rng.hash4(99, 7, a, b)) == orc.hash4(99, 7, a, b)
        assert int(rng.uniform_int(rng.hash4(3, 1, a, b), 1, 6)) == orc.uniform_int(orc.hash4(3, 1, a, b), 1, 6)


def test_uniform_ranges_and_means():
    h = rng.hash4(1, 2, 0, np.arange(200000, dtype=np.uint64))
    u = rng.uniform01_f32(h)
    assert u.min() >= 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.005
    k = rng.uniform_int(h, 0, 4)
    assert set(np.unique(k)) == {0, 1, 2, 3, 4}
    assert np.allclose(np.bincount(k) / len(k), 0.2, atol=0.005)
    b = rng.bernoulli(h, rng.BERNOULLI_0_1)
    assert abs(b.mean() - 0.1) < 0.003


def test_irwin_hall_moments():
    v = rng.irwin_hall12_f32(5, 0, np.arange(100000, dtype=np.uint64))
    assert abs(v.mean()) < 0.02 and abs(v.std() - 1.0) < 0.02
    assert v.min() >= -6 and v.max() <= 6


def test_micro_inputs_shape():
    inp = W.micro_inputs(65536, 10)
    assert inp.x0.shape == (65536,) and inp.xs.shape == (10, 21846)
    assert inp.x0.dtype == np.float32 and inp.vs.dtype == np.float32


def test_world_sides_log_uniform():
    s = W.world_sides(256)
    assert s.min() >= 64 and s.max() <= 1024
    total = int((s.astype(np.int64) ** 2).sum())
    assert 30e6 < total < 70e6                    # expectation ~48.2 M cells


def test_sugar_inputs_counts():
    inp = W.sugar_inputs(128, 4096)
    assert int(inp.occ.sum()) == 4096
    m = inp.occ.astype(bool)
    assert inp.a_sugar[m].min() >= 5 and inp.a_sugar[m].max() <= 25
    assert (inp.a_sugar[~m] == 0).all()
    assert np.array_equal(inp.sugar, inp.cap)
