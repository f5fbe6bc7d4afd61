"""Seeded synthetic inputs for the five workloads.

Each generator returns plain numpy arrays and sizes; nothing here computes
any part of the method (allocation, enumeration, or the simulations).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import rng

# ---------------------------------------------------------------- micro ----


@dataclass
class MicroInputs:
    n_init: int          # objects created at start, ids 0..n_init-1
    steps: int           # update / cull / re-new rounds
    n_renew: int         # ids 3k, k < n_renew, re-created each step
    x0: np.ndarray       # float32 [n_init]
    v0: np.ndarray       # float32 [n_init]
    xs: np.ndarray       # float32 [steps, n_renew]  x of the re-created id 3k
    vs: np.ndarray       # float32 [steps, n_renew]


def micro_inputs(n_init: int = 65536, steps: int = 10,
                 seed: int = rng.DEFAULT_SEED) -> MicroInputs:
    ids = np.arange(n_init, dtype=np.uint64)
    x0 = rng.uniform01_f32(rng.hash4(seed, rng.S_MICRO_X, 0, ids))
    v0 = rng.irwin_hall12_f32(seed, 0, ids)
    n_renew = (n_init + 2) // 3
    rid = (3 * np.arange(n_renew, dtype=np.uint64))[None, :]
    st = np.arange(1, steps + 1, dtype=np.uint64)[:, None]
    xs = rng.uniform01_f32(rng.hash4(seed, rng.S_MICRO_X, st, rid))
    vs = rng.irwin_hall12_f32(seed, st, rid)
    return MicroInputs(n_init, steps, n_renew, x0, v0,
                       np.ascontiguousarray(xs, dtype=np.float32),
                       np.ascontiguousarray(vs, dtype=np.float32))


# ----------------------------------------------------------- game of life --


def gol_grid(width: int, height: int, seed: int = rng.DEFAULT_SEED,
             threshold24: int = rng.BERNOULLI_0_1) -> np.ndarray:
    """uint8 [height, width]; cell (x, y) is alive with probability ~0.1."""
    p = np.arange(width * height, dtype=np.uint64)
    alive = rng.bernoulli(rng.hash4(seed, rng.S_GOL_ALIVE, 0, p), threshold24)
    return alive.astype(np.uint8).reshape(height, width)


# ------------------------------------------------------------- batched -----


def world_sides(n_worlds: int = 256, lo: int = 64, hi: int = 1024,
                seed: int = rng.DEFAULT_SEED) -> np.ndarray:
    """Square world sides, log-uniform in [lo, hi]: round(lo * (hi/lo)**u)."""
    w = np.arange(n_worlds, dtype=np.uint64)
    u = rng.uniform01_f32(rng.hash4(seed, rng.S_WORLD_SIZE, 0, w)).astype(np.float64)
    sides = np.rint(lo * (hi / lo) ** u).astype(np.int64)
    return np.clip(sides, lo, hi).astype(np.int32)


def world_seeds(n_worlds: int, seed: int = rng.DEFAULT_SEED) -> np.ndarray:
    w = np.arange(n_worlds, dtype=np.uint64)
    return rng.hash4(seed, rng.S_WORLD_SEED, 0, w).astype(np.uint64)


@dataclass
class BatchInputs:
    sides: np.ndarray          # int32 [n_worlds]
    seeds: np.ndarray          # uint64 [n_worlds]
    grids: list                # uint8 [side, side] per world
    generations: int


def batch_inputs(n_worlds: int = 256, generations: int = 100, lo: int = 64,
                 hi: int = 1024, seed: int = rng.DEFAULT_SEED) -> BatchInputs:
    sides = world_sides(n_worlds, lo, hi, seed)
    seeds = world_seeds(n_worlds, seed)
    grids = [gol_grid(int(s), int(s), int(ws)) for s, ws in zip(sides, seeds)]
    return BatchInputs(sides, seeds, grids, generations)


# ------------------------------------------------------------ sugarscape ---

# Rule constants of the Sugarscape-style model (agents die at max_age;
# reproduce with at least repro_min sugar while fertile_min <= age <= fertile_max).
SUGAR_RULES = dict(max_age=100, repro_min=20, fertile_min=10, fertile_max=60)


@dataclass
class SugarInputs:
    side: int
    n_agents: int
    seed: int
    sugar: np.ndarray      # int32 [side*side]  (starts equal to cap)
    cap: np.ndarray        # int32 [side*side]  U{0..4}
    occ: np.ndarray        # uint8 [side*side]
    a_sugar: np.ndarray    # int32 [side*side]  U{5..25} where occupied, else 0
    a_metab: np.ndarray    # U{1..4}
    a_vision: np.ndarray   # U{1..6}
    a_age: np.ndarray      # U{0..max_age-1}


def sugar_inputs(side: int = 2048, n_agents: int = 1 << 20, seed: int = rng.DEFAULT_SEED,
                 max_age: int = SUGAR_RULES["max_age"]) -> SugarInputs:
    n = side * side
    if not 0 <= n_agents <= n:
        raise ValueError("n_agents must fit on the grid")
    cells = np.arange(n, dtype=np.uint64)
    cap = rng.uniform_int(rng.hash4(seed, rng.S_SUGAR_CAP, 0, cells), 0, 4)
    key = rng.hash4(seed, rng.S_SUGAR_OCC, 0, cells)
    order = np.lexsort((cells, key))       # by key, ties by cell index
    occ = np.zeros(n, dtype=np.uint8)
    occ[order[:n_agents]] = 1
    m = occ.astype(bool)

    def trait(stream, lo, hi):
        v = rng.uniform_int(rng.hash4(seed, stream, 0, cells), lo, hi)
        return np.where(m, v, 0).astype(np.int32)

    return SugarInputs(side, n_agents, seed, cap.copy(), cap, occ,
                       trait(rng.S_SUGAR_SUGAR, 5, 25), trait(rng.S_SUGAR_METAB, 1, 4),
                       trait(rng.S_SUGAR_VISION, 1, 6), trait(rng.S_SUGAR_AGE, 0, max_age - 1))


# ---------------------------------------------------------------- serving ---


@dataclass
class EpisodeSpec:
    eid: int
    kind: str          # "gol" or "sugar"
    side: int
    length: int        # generations (gol) or steps (sugar)
    seed: int
    agents: int        # sugar only
    arrival: float     # seconds after the start of the run


def serving_episodes(n: int, rate: float, seed: int = rng.DEFAULT_SEED, gol_frac: float = 0.7,
                     gol_sides=(128, 2048), gol_lengths=(50, 300), sugar_sides=(256, 1024),
                     sugar_agents=(10_000, 200_000), sugar_steps: int = 100) -> list:
    """Episodes with Poisson arrivals (rate per second; inf = all at time 0):
    70% Game of Life (side log-uniform, generations uniform), 30% Sugarscape
    (side log-uniform, agents uniform, capped at a quarter of the cells)."""
    e = np.arange(n, dtype=np.uint64)
    h = lambda k: rng.hash4(seed, rng.S_EPISODE, k, e)
    kind = rng.uniform01_f32(h(0)) < gol_frac
    u = rng.uniform01_f32(h(1)).astype(np.float64)
    gl = rng.uniform_int(h(2), *gol_lengths)
    ag = rng.uniform_int(h(3), *sugar_agents)
    ia = rng.uniform01_f32(h(4)).astype(np.float64)
    seeds = h(5)
    out, t = [], 0.0
    for i in range(n):
        if np.isfinite(rate):
            t += -np.log(1.0 - ia[i]) / rate
        if kind[i]:
            lo, hi = gol_sides
            side = int(np.rint(lo * (hi / lo) ** u[i]))
            out.append(EpisodeSpec(i, "gol", side, int(gl[i]), int(seeds[i]), 0, t))
        else:
            lo, hi = sugar_sides
            side = int(np.rint(lo * (hi / lo) ** u[i]))
            out.append(EpisodeSpec(i, "sugar", side, sugar_steps, int(seeds[i]),
                                   min(int(ag[i]), side * side // 4), t))
    return out


def episode_inputs(ep: EpisodeSpec):
    """Initial state of an episode (a GoL grid or Sugarscape inputs)."""
    if ep.kind == "gol":
        return gol_grid(ep.side, ep.side, seed=ep.seed)
    return sugar_inputs(ep.side, ep.agents, seed=ep.seed)


# ---------------------------------------------------------------- traffic --

# Nagel-Schreckenberg constants: top speed, slowdown and entry probabilities
# as 24-bit Bernoulli thresholds.
TRAFFIC_RULES = dict(vmax=5, p_slow24=1 << 22, p_in24=1 << 23)  # p_slow 0.25, p_in 0.5
TRAFFIC_DENSITY24 = 2516582  # floor(0.15 * 2**24)


@dataclass
class TrafficInputs:
    roads: int
    length: int
    seed: int
    vel: np.ndarray   # int32 [roads, length]: a car's speed, -1 = empty cell


def traffic_inputs(roads: int = 1024, length: int = 1024, seed: int = rng.DEFAULT_SEED,
                   density24: int = TRAFFIC_DENSITY24, vmax: int = 5) -> TrafficInputs:
    """Roads of `length` cells; cell (r, i) holds a car with probability
    density24 / 2**24 and the car's speed is U{0..vmax}."""
    r = np.arange(roads, dtype=np.uint64)[:, None]
    i = np.arange(length, dtype=np.uint64)[None, :]
    occ = rng.bernoulli(rng.hash4(seed, rng.S_TRAFFIC_OCC, r, i), density24)
    v0 = rng.uniform_int(rng.hash4(seed, rng.S_TRAFFIC_V0, r, i), 0, vmax)
    vel = np.where(occ, v0, -1).astype(np.int32)
    return TrafficInputs(roads, length, seed, np.ascontiguousarray(vel))


# ------------------------------------------------------------- collisions --

# Time step, softening and merge radius squared (float32 values).
COLLIDE_PARAMS = dict(dt=0.01, eps2=0.01, r2_merge=0.0001)


@dataclass
class CollideInputs:
    n: int
    seed: int
    x: np.ndarray
    y: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    m: np.ndarray


def collide_inputs(n: int = 4096, seed: int = rng.DEFAULT_SEED, box: float = 8.0) -> CollideInputs:
    """n bodies uniform in [0, box)^2, velocities uniform in [-0.5, 0.5)^2,
    masses U{1..4} / 1024 (all values exact in float32)."""
    i = np.arange(n, dtype=np.uint64)
    x = (rng.uniform01_f32(rng.hash4(seed, rng.S_BODY_X, 0, i)) * np.float32(box)).astype(np.float32)
    y = (rng.uniform01_f32(rng.hash4(seed, rng.S_BODY_Y, 0, i)) * np.float32(box)).astype(np.float32)
    vx = (rng.uniform01_f32(rng.hash4(seed, rng.S_BODY_VX, 0, i)) - np.float32(0.5)).astype(np.float32)
    vy = (rng.uniform01_f32(rng.hash4(seed, rng.S_BODY_VY, 0, i)) - np.float32(0.5)).astype(np.float32)
    m = (rng.uniform_int(rng.hash4(seed, rng.S_BODY_M, 0, i), 1, 4).astype(np.float32) *
         np.float32(1.0 / 1024)).astype(np.float32)
    return CollideInputs(n, seed, x, y, vx, vy, m)



# ------------------------------------------------------------------ wa-tor --

WATOR_RULES = dict(fish_breed=3, shark_breed=10, starve=3)
WATOR_FISH24 = 5033164   # floor(0.30 * 2**24)
WATOR_SHARK24 = 838860   # floor(0.05 * 2**24)


@dataclass
class WatorInputs:
    side: int
    seed: int
    kind: np.ndarray     # int32 [side, side]: 0 empty, 1 fish, 2 shark
    age: np.ndarray      # int32 [side, side]
    energy: np.ndarray   # int32 [side, side]


def wator_inputs(side: int = 1024, seed: int = rng.DEFAULT_SEED, rules: dict = WATOR_RULES,
                 fish24: int = WATOR_FISH24, shark24: int = WATOR_SHARK24) -> WatorInputs:
    """Each cell holds a fish with probability fish24 / 2**24, else a shark
    with probability shark24 / 2**24 (one 24-bit draw); fish ages
    U{0..fish_breed-1}, shark ages U{0..shark_breed-1}, shark energies
    U{1..starve}."""
    c = np.arange(side * side, dtype=np.uint64).reshape(side, side)
    u = (rng.hash4(seed, rng.S_WATOR_KIND, 0, c) >> np.uint64(40)).astype(np.int64)
    kind = np.where(u < fish24, 1, np.where(u < fish24 + shark24, 2, 0)).astype(np.int32)
    fa = rng.uniform_int(rng.hash4(seed, rng.S_WATOR_FISH_AGE, 0, c), 0, rules["fish_breed"] - 1)
    sa = rng.uniform_int(rng.hash4(seed, rng.S_WATOR_SHARK_AGE, 0, c), 0, rules["shark_breed"] - 1)
    se = rng.uniform_int(rng.hash4(seed, rng.S_WATOR_ENERGY, 0, c), 1, rules["starve"])
    age = np.where(kind == 1, fa, np.where(kind == 2, sa, 0)).astype(np.int32)
    energy = np.where(kind == 2, se, 0).astype(np.int32)
    return WatorInputs(side, seed, np.ascontiguousarray(kind), np.ascontiguousarray(age),
                       np.ascontiguousarray(energy))
