"""CPU oracle for the SMMO object heap and parallel do-all (arXiv 1809.07444).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain sequential C library
(``oracle.c``) plus this ctypes wrapper.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product package
never does, and the two share no code.

Functions follow the paper's sections:
  * hierarchical bitmap model: Sec. 2.1 (operations), Sec. 3 (data structure,
    container consistency, Alg. 2), with a container-width parameter so the
    width-4 example figure of Sec. 3 can be replayed;
  * heap model: Sec. 2 (block states), Sec. 2.2 (Alg. 1);
  * workloads: the microbenchmark (per-object definition), Game of Life
    (dense B3/S23 torus) and the Sugarscape-style rules spelled out in
    ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

i32, i64, u64, f32p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float)
vp = ctypes.c_void_p


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_mix64.restype = u64
        L.orc_mix64.argtypes = [u64]
        L.orc_hash.restype = u64
        L.orc_hash.argtypes = [u64, u64, u64, u64]
        L.orc_uniform_int.restype = i32
        L.orc_uniform_int.argtypes = [u64, i32, i32]
        L.orc_bm_new.restype = vp
        L.orc_bm_new.argtypes = [i64, ctypes.c_int, ctypes.c_int]
        L.orc_bm_delete.argtypes = [vp]
        L.orc_bm_nlevels.restype = ctypes.c_int
        L.orc_bm_nlevels.argtypes = [vp]
        L.orc_bm_nwords.restype = i64
        L.orc_bm_nwords.argtypes = [vp, ctypes.c_int]
        L.orc_bm_words.argtypes = [vp, ctypes.c_int, vp]
        L.orc_bm_trace.restype = i64
        L.orc_bm_trace.argtypes = [vp, vp, i64]
        L.orc_bm_op.restype = ctypes.c_int
        L.orc_bm_op.argtypes = [vp, ctypes.c_int, i64, ctypes.POINTER(i64)]
        L.orc_type_capacity.restype = i32
        L.orc_type_capacity.argtypes = [vp, i32, i32]
        L.orc_visit_types.restype = ctypes.c_uint32
        L.orc_visit_types.argtypes = [vp, i32, i32]
        L.orc_heap_new.restype = vp
        L.orc_heap_new.argtypes = [i32, i32, i32]
        L.orc_heap_delete.argtypes = [vp]
        L.orc_heap_alloc.restype = i64
        L.orc_heap_alloc.argtypes = [vp, i32]
        L.orc_heap_free.restype = ctypes.c_int
        L.orc_heap_free.argtypes = [vp, i64]
        L.orc_heap_reclaim.restype = i64
        L.orc_heap_reclaim.argtypes = [vp]
        L.orc_heap_check.restype = i64
        L.orc_heap_check.argtypes = [vp]
        L.orc_heap_counts.argtypes = [vp, vp]
        L.orc_heap_dump.argtypes = [vp, vp, vp]
        L.orc_micro_run.restype = ctypes.c_int
        L.orc_micro_run.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_gol_step.restype = ctypes.c_int
        L.orc_gol_step.argtypes = [i32, i32, vp, vp, vp]
        L.orc_gol_run.restype = ctypes.c_int
        L.orc_gol_run.argtypes = [i32, i32, i32, vp, vp]
        L.orc_sugar_run.restype = ctypes.c_int
        L.orc_sugar_run.argtypes = [i32, i32, i32, u64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_collide_run.restype = ctypes.c_int
        L.orc_collide_run.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.orc_traffic_run.restype = ctypes.c_int
        L.orc_traffic_run.argtypes = [i32, i32, i32, i32, u64, i32, ctypes.c_uint32, ctypes.c_uint32, vp, vp]
        L.orc_wator_run.restype = ctypes.c_int
        L.orc_wator_run.argtypes = [i32, i32, i32, u64, i32, i32, i32, vp, vp, vp, vp]
        _lib = L
    return _lib


def type_capacity(sizes, t: int) -> int:
    """Slots per block of type t (Sec. 2 byte-size rule) among types of the given byte sizes."""
    a = np.ascontiguousarray(sizes, dtype=np.int32)
    return int(lib().orc_type_capacity(a.ctypes.data_as(ctypes.c_void_p), len(a), t))


def visit_types(parents, t: int) -> set:
    """Types a do-all over type t visits (t and every type inheriting from
    it); parents[u] is u's parent index or None.  Empty set if the parent
    links are not a forest."""
    a = np.array([-1 if p is None else p for p in parents], dtype=np.int32)
    m = int(lib().orc_visit_types(a.ctypes.data_as(ctypes.c_void_p), len(a), t))
    return {u for u in range(len(a)) if m >> u & 1}


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------------- RNG ---

def mix64(z: int) -> int:
    return int(lib().orc_mix64(z))


def hash4(seed: int, stream: int, a: int, b: int) -> int:
    return int(lib().orc_hash(seed, stream, a, b))


def uniform_int(h: int, lo: int, hi: int) -> int:
    return int(lib().orc_uniform_int(h, lo, hi))


# ------------------------------------------------------ bitmap model -------

OP_TRY_SET, OP_TRY_CLEAR, OP_SET, OP_CLEAR, OP_TRY_FIND_SET, OP_FIND_CLEAR, OP_GET = range(7)
FAIL = -1


class Bitmap:
    """Sequential hierarchical bitmap (Sec. 3) with container width ``width``."""

    def __init__(self, nbits: int, width: int = 64, all_set: bool = False):
        self._h = lib().orc_bm_new(nbits, width, 1 if all_set else 0)
        if not self._h:
            raise ValueError("bad bitmap geometry")
        self.nbits = nbits
        self.width = width

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_bm_delete(self._h)
            self._h = None

    def _op(self, op: int, pos: int = 0) -> int:
        r = i64(0)
        if lib().orc_bm_op(self._h, op, pos, ctypes.byref(r)) != 0:
            raise IndexError(pos)
        return int(r.value)

    def try_set(self, pos): return bool(self._op(OP_TRY_SET, pos))
    def try_clear(self, pos): return bool(self._op(OP_TRY_CLEAR, pos))
    def set(self, pos): return self._op(OP_SET, pos) == 0
    def clear(self, pos): return self._op(OP_CLEAR, pos) == 0
    def try_find_set(self): return self._op(OP_TRY_FIND_SET)
    def find_clear(self): return self._op(OP_FIND_CLEAR)
    def get(self, pos): return bool(self._op(OP_GET, pos))

    @property
    def nlevels(self) -> int:
        return int(lib().orc_bm_nlevels(self._h))

    def words(self, level: int) -> np.ndarray:
        n = int(lib().orc_bm_nwords(self._h, level))
        out = np.zeros(n, dtype=np.uint64)
        lib().orc_bm_words(self._h, level, _p(out))
        return out

    def trace(self) -> list[tuple[int, int]]:
        """Every successful clear so far as (level, position), in order."""
        n = int(lib().orc_bm_trace(self._h, None, 0))
        out = np.zeros(max(n, 1), dtype=np.int64)
        lib().orc_bm_trace(self._h, _p(out), n)
        return [(int(v) >> 40, int(v) & ((1 << 40) - 1)) for v in out[:n]]


# ---------------------------------------------------------- heap model -----

MAX_TYPES = 8
CHECK_BITS = {1: "I2", 2: "I3", 3: "I4", 4: "I5", 5: "I6", 6: "I7"}


class HeapModel:
    """Sequential Alg. 1 heap: lowest active block, lowest slot, lowest free block."""

    def __init__(self, num_blocks: int, capacity: int = 64, num_types: int = 1):
        self._h = lib().orc_heap_new(num_blocks, capacity, num_types)
        if not self._h:
            raise ValueError("bad heap geometry")
        self.num_blocks, self.capacity, self.num_types = num_blocks, capacity, num_types

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_heap_delete(self._h)
            self._h = None

    def alloc(self, t: int = 0) -> int:
        return int(lib().orc_heap_alloc(self._h, t))

    def free(self, handle: int) -> bool:
        return lib().orc_heap_free(self._h, handle) == 0

    def reclaim(self) -> int:
        return int(lib().orc_heap_reclaim(self._h))

    def check(self) -> list[str]:
        bits = int(lib().orc_heap_check(self._h))
        return [name for b, name in CHECK_BITS.items() if bits >> b & 1]

    def counts(self) -> dict:
        out = np.zeros(1 + 5 * MAX_TYPES, dtype=np.int64)
        lib().orc_heap_counts(self._h, _p(out))
        d = {"free_blocks": int(out[0])}
        for t in range(self.num_types):
            a = out[1 + 5 * t: 6 + 5 * t]
            d[t] = dict(allocated_blocks=int(a[0]), active_blocks=int(a[1]), live=int(a[2]),
                        allocs=int(a[3]), frees=int(a[4]))
        return d

    def dump(self):
        ob = np.zeros(self.num_blocks, dtype=np.uint64)
        bt = np.zeros(self.num_blocks, dtype=np.int32)
        lib().orc_heap_dump(self._h, _p(ob), _p(bt))
        return ob, bt


# --------------------------------------------------------------- micro -----

@dataclass
class MicroResult:
    x: np.ndarray
    v: np.ndarray
    present: np.ndarray
    allocs: int
    frees: int


def micro_run(inp) -> MicroResult:
    """Reference for the microbenchmark: ``inp`` is synth.workloads.MicroInputs."""
    n = inp.n_init
    x = np.zeros(n, dtype=np.float32)
    v = np.zeros(n, dtype=np.float32)
    pres = np.zeros(n, dtype=np.uint8)
    counts = np.zeros(2, dtype=np.int64)
    x0 = np.ascontiguousarray(inp.x0, dtype=np.float32)
    v0 = np.ascontiguousarray(inp.v0, dtype=np.float32)
    xs = np.ascontiguousarray(inp.xs, dtype=np.float32)
    vs = np.ascontiguousarray(inp.vs, dtype=np.float32)
    rc = lib().orc_micro_run(n, inp.steps, inp.n_renew, _p(x0), _p(v0), _p(xs), _p(vs),
                             _p(x), _p(v), _p(pres), _p(counts))
    if rc != 0:
        raise ValueError("micro_run: bad arguments")
    return MicroResult(x, v, pres, int(counts[0]), int(counts[1]))


# --------------------------------------------------------- game of life ----

def gol_step(grid: np.ndarray):
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    h, w = g.shape
    out = np.zeros_like(g)
    counts = np.zeros(4, dtype=np.int64)
    lib().orc_gol_step(w, h, _p(g), _p(out), _p(counts))
    return out, counts


def gol_run(grid: np.ndarray, generations: int):
    """Returns (final grid, counts[generations, 4]) with columns
    (candidates, births, deaths, population after the generation)."""
    g = np.array(grid, dtype=np.uint8, order="C", copy=True)
    h, w = g.shape
    counts = np.zeros((max(generations, 1), 4), dtype=np.int64)
    rc = lib().orc_gol_run(w, h, generations, _p(g), _p(counts))
    if rc != 0:
        raise ValueError("gol_run: bad arguments")
    return g, counts[:generations]


# ------------------------------------------------------------ sugarscape ---

class _Rules(ctypes.Structure):
    _fields_ = [("max_age", i32), ("repro_min", i32), ("fertile_min", i32), ("fertile_max", i32)]


@dataclass
class SugarState:
    side: int
    sugar: np.ndarray      # int32 [side*side]
    cap: np.ndarray        # int32 [side*side]
    occ: np.ndarray        # uint8 [side*side]
    a_sugar: np.ndarray    # int32 [side*side], valid where occ
    a_metab: np.ndarray
    a_vision: np.ndarray
    a_age: np.ndarray
    births: int = 0
    deaths: int = 0
    moves: int = 0

    def copy(self) -> "SugarState":
        return SugarState(self.side, self.sugar.copy(), self.cap.copy(), self.occ.copy(),
                          self.a_sugar.copy(), self.a_metab.copy(), self.a_vision.copy(),
                          self.a_age.copy(), self.births, self.deaths, self.moves)


def sugar_run(state: SugarState, steps: int, seed: int, rules: dict, step0: int = 0) -> SugarState:
    """Advances a copy of ``state`` by ``steps`` synchronous steps."""
    s = state.copy()
    r = _Rules(rules["max_age"], rules["repro_min"], rules["fertile_min"], rules["fertile_max"])
    counts = np.array([s.births, s.deaths, s.moves], dtype=np.int64)
    rc = lib().orc_sugar_run(s.side, steps, step0, seed, ctypes.byref(r), _p(s.sugar), _p(s.cap),
                             _p(s.occ), _p(s.a_sugar), _p(s.a_metab), _p(s.a_vision), _p(s.a_age),
                             _p(counts))
    if rc != 0:
        raise ValueError("sugar_run: bad arguments")
    s.births, s.deaths, s.moves = (int(c) for c in counts)
    return s


@dataclass
class TrafficResult:
    vel: np.ndarray      # int32 [roads, length], -1 = empty
    entries: int
    exits: int


def traffic_run(vel: np.ndarray, steps: int, seed: int, rules: dict, step0: int = 0) -> TrafficResult:
    """Nagel-Schreckenberg traffic (open roads) from the speed grid `vel`."""
    v = np.ascontiguousarray(vel, dtype=np.int32).copy()
    counts = np.zeros(2, dtype=np.int64)
    roads, length = v.shape
    rc = lib().orc_traffic_run(roads, length, steps, step0, seed, rules["vmax"], rules["p_slow24"],
                               rules["p_in24"], _p(v), _p(counts))
    if rc != 0:
        raise ValueError("orc_traffic_run failed")
    return TrafficResult(v, int(counts[0]), int(counts[1]))


class _CollideParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("eps2", ctypes.c_float), ("r2_merge", ctypes.c_float)]


@dataclass
class CollideState:
    x: np.ndarray
    y: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    m: np.ndarray      # 0 = merged away
    merges: int = 0


def collide_run(state: CollideState, steps: int, params: dict) -> CollideState:
    """Merging-bodies particle system (float32, every operation rounded once)."""
    a = [np.ascontiguousarray(v, dtype=np.float32).copy() for v in (state.x, state.y, state.vx, state.vy, state.m)]
    counts = np.zeros(1, dtype=np.int64)
    pr = _CollideParams(params["dt"], params["eps2"], params["r2_merge"])
    rc = lib().orc_collide_run(len(a[0]), steps, ctypes.byref(pr), *[_p(v) for v in a], _p(counts))
    if rc != 0:
        raise ValueError("orc_collide_run failed")
    return CollideState(*a, merges=state.merges + int(counts[0]))



@dataclass
class WatorState:
    kind: np.ndarray     # int32 [side, side]: 0 empty, 1 fish, 2 shark
    age: np.ndarray      # int32 [side, side]
    energy: np.ndarray   # int32 [side, side], sharks
    fish_born: int = 0
    sharks_born: int = 0
    fish_eaten: int = 0
    sharks_starved: int = 0

    def copy(self) -> "WatorState":
        return WatorState(self.kind.copy(), self.age.copy(), self.energy.copy(), self.fish_born,
                          self.sharks_born, self.fish_eaten, self.sharks_starved)


def wator_run(state: WatorState, steps: int, seed: int, rules: dict, step0: int = 0) -> WatorState:
    """Wa-Tor (fish and sharks) for `steps` steps from step index step0; counts accumulate."""
    s = state.copy()
    s.kind = np.ascontiguousarray(s.kind, dtype=np.int32)
    s.age = np.ascontiguousarray(s.age, dtype=np.int32)
    s.energy = np.ascontiguousarray(s.energy, dtype=np.int32)
    counts = np.zeros(4, dtype=np.int64)
    side = s.kind.shape[0]
    rc = lib().orc_wator_run(side, steps, step0, seed, rules["fish_breed"], rules["shark_breed"], rules["starve"],
                             _p(s.kind), _p(s.age), _p(s.energy), _p(counts))
    if rc != 0:
        raise ValueError("orc_wator_run failed")
    s.fish_born += int(counts[0])
    s.sharks_born += int(counts[1])
    s.fish_eaten += int(counts[2])
    s.sharks_starved += int(counts[3])
    return s
