"""Counter-based random numbers for the synthetic workloads.

Every random quantity in the workloads is a pure function of
(seed, stream, a, b), so any element can be drawn independently, in any
order, on any device.  The mixing function is the SplitMix64 output
finaliser (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; public-domain reference code by S. Vigna):

    mix64(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
              z ^= z >> 27; z *= 0x94D049BB133111EB;
              z ^= z >> 31                                  (mod 2**64)

    hash(seed, stream, a, b) =
        mix64(mix64(mix64(seed ^ stream * 0x9E3779B97F4A7C15) ^ a) ^ b)

Derived draws (all exact, integer-only until the final float):
    U[0,1)          = (h >> 40) * 2**-24                 (exact in float32)
    U{lo..hi}       = lo + (((h >> 32) * (hi - lo + 1)) >> 32)
    Bernoulli(p)    = (h >> 40) < floor(p * 2**24)
    N(0,1) stand-in = ((u_0 + u_1) + ... + u_11) - 6   (Irwin-Hall, twelve
                      float32 uniforms summed left to right in float32)

This module holds no arithmetic of the method itself: it only produces the
seeded inputs that both the device path and the oracle consume.
"""
from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

# Stream tags, one per kind of draw.
S_MICRO_X = 1
S_GOL_ALIVE = 3
S_SUGAR_CAP = 4
S_SUGAR_OCC = 5
S_SUGAR_SUGAR = 6
S_SUGAR_METAB = 7
S_SUGAR_VISION = 8
S_SUGAR_AGE = 9
S_SUGAR_CHILD_METAB = 10
S_SUGAR_CHILD_VISION = 11
S_WORLD_SIZE = 12
S_WORLD_SEED = 13
S_WORLD_KIND = 14
S_EPISODE = 15
S_MICRO_V0 = 16  # 16..27: the twelve Irwin-Hall sub-streams
S_TRAFFIC_OCC = 30
S_TRAFFIC_V0 = 31
S_TRAFFIC_SLOW = 32   # drawn by the method itself, each step (both sides implement hash)
S_TRAFFIC_IN = 33     # idem
S_BODY_X = 34
S_BODY_Y = 35
S_BODY_VX = 36
S_BODY_VY = 37
S_BODY_M = 38
S_WATOR_FISH = 40    # drawn by the method itself, each step (both sides implement hash)
S_WATOR_SHARK = 41   # idem
S_WATOR_KIND = 42
S_WATOR_FISH_AGE = 43
S_WATOR_SHARK_AGE = 44
S_WATOR_ENERGY = 45

DEFAULT_SEED = 24301
BERNOULLI_0_1 = 1677721  # floor(0.1 * 2**24)


def _u64(x) -> np.ndarray:
    return np.asarray(x, dtype=np.uint64)


def mix64(z) -> np.ndarray:
    z = _u64(z).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def hash4(seed: int, stream: int, a, b) -> np.ndarray:
    """hash(seed, stream, a, b) as defined in the module docstring.

    ``a`` and ``b`` broadcast against each other (uint64 arrays or ints)."""
    s = (int(seed) ^ ((int(stream) * GOLDEN) & MASK64)) & MASK64
    h0 = mix64(np.uint64(s))
    a = _u64(a)
    b = _u64(b)
    h1 = mix64(h0 ^ a)
    return mix64(h1 ^ b)


def uniform01_f32(h) -> np.ndarray:
    """U[0,1) with 24 random bits, exactly representable in float32."""
    top = (_u64(h) >> np.uint64(40)).astype(np.float64)
    return (top * 2.0 ** -24).astype(np.float32)


def uniform_int(h, lo: int, hi: int) -> np.ndarray:
    span = np.uint64(hi - lo + 1)
    with np.errstate(over="ignore"):
        v = ((_u64(h) >> np.uint64(32)) * span) >> np.uint64(32)
    return (v.astype(np.int64) + lo).astype(np.int32)


def bernoulli(h, threshold24: int) -> np.ndarray:
    return (_u64(h) >> np.uint64(40)) < np.uint64(threshold24)


def irwin_hall12_f32(seed: int, step, ids) -> np.ndarray:
    """N(0,1) stand-in: twelve float32 uniforms summed left to right, minus 6."""
    acc = None
    for k in range(12):
        u = uniform01_f32(hash4(seed, S_MICRO_V0 + k, step, ids))
        acc = u if acc is None else (acc + u).astype(np.float32)
    return (acc - np.float32(6.0)).astype(np.float32)


def splitmix64_sequence(state: int, n: int) -> list[int]:
    """The published SplitMix64 generator (state += golden; output mix64(state)).

    Only used to pin mix64 against the generator's reference output."""
    out = []
    for _ in range(n):
        state = (state + GOLDEN) & MASK64
        out.append(int(mix64(np.uint64(state))))
    return out
