"""Host drivers of the workloads over the C ABI (argument marshalling only)."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi as C
from .heap import Heap

MICRO_TYPE = (4, 4, 4)  # {int32 id, float32 x, float32 v}


@dataclass
class MicroGpuResult:
    x: np.ndarray
    v: np.ndarray
    present: np.ndarray
    stats: dict


class MicroBench:
    """The alloc/do-all microbenchmark on one heap, inputs resident on the device."""

    def __init__(self, inp, num_blocks: int = 4096, capacity: int = 64, flags: int = C.DO_PERSISTENT,
                 device="cuda"):
        self.inp = inp
        self.flags = flags
        self.heap = Heap(num_blocks, capacity, [MICRO_TYPE], device=device)
        self.x0 = torch.from_numpy(np.ascontiguousarray(inp.x0)).to(device)
        self.v0 = torch.from_numpy(np.ascontiguousarray(inp.v0)).to(device)
        self.xs = torch.from_numpy(np.ascontiguousarray(inp.xs)).to(device)
        self.vs = torch.from_numpy(np.ascontiguousarray(inp.vs)).to(device)
        self.lib = self.heap.lib

    def init(self):
        h = self.heap
        C.check(self.lib.dsoar_micro_init(h.h, 0, self.inp.n_init, self.x0.data_ptr(), self.v0.data_ptr(),
                                          h._s()), "dsoar_micro_init")

    def step(self, s: int):
        h = self.heap
        n = self.inp.n_renew
        C.check(self.lib.dsoar_micro_step(h.h, 0, n, self.xs[s].data_ptr(), self.vs[s].data_ptr(),
                                          self.flags, h._s()), "dsoar_micro_step")

    def run(self):
        self.heap.reset()
        self.init()
        for s in range(self.inp.steps):
            self.step(s)

    def result(self) -> MicroGpuResult:
        n = self.inp.n_init
        x, px = self.heap.gather(0, 0, 1, n)
        v, pv = self.heap.gather(0, 0, 2, n)
        torch.cuda.synchronize()
        return MicroGpuResult(x.cpu().numpy().view(np.float32), v.cpu().numpy().view(np.float32),
                              px.cpu().numpy(), self.heap.stats(raise_sticky=False))


def micro_run(inp, num_blocks: int = 4096, capacity: int = 64, flags: int = C.DO_PERSISTENT) -> MicroGpuResult:
    mb = MicroBench(inp, num_blocks, capacity, flags)
    mb.run()
    return mb.result()


# ------------------------------------------------------------ game of life --

GOL_TYPES = [(4,), (4, 4, 4), (4, 4, 4)]  # Cell, Alive, Candidate
GOL_CELL, GOL_ALIVE, GOL_CAND = 0, 1, 2


def gol_blocks_for(total_cells: int, capacity: int = 64) -> int:
    """Heap size for a Game of Life state: one block per `capacity` cells for
    the Cells and twice as many again for Alive and Candidate objects (at most
    one of them per cell, plus partly filled blocks), rounded up to a multiple
    of 4096 blocks (64 level-0 bitmap words).  Not to a power of two: every
    enumeration scans the whole allocated bitmap, so a heap no larger than
    this rule asks for keeps that scan short.  Capacity 0 (per-type
    capacities by object size): Cells {4 B} have 64 slots, Alive and
    Candidate {3 x 4 B} 16."""
    if capacity == 0:
        need = max(64, -(-total_cells // 64) + 2 * -(-total_cells // 16))
    else:
        need = max(64, 3 * -(-total_cells // capacity))
    return -(-need // 4096) * 4096


class GameOfLife:
    """One or many square Game-of-Life worlds as objects in one device heap."""

    # Every generation creates its Candidates in bulk (several blocks per
    # wavefront) into a type with no active blocks: whole free blocks first
    # is faster than the dense policy here (about 20 against 30 ms for 200
    # generations of 1024^2 on MI355X) and gives the same results.
    BULK_MIN = 0
    # Candidates all die within their generation: they skip the active lookup
    # and each wavefront opens blocks of its own (12.5 against 13.7 ms for
    # 200 generations of 1024^2 on MI355X, same results).
    CAND_POLICY = C.POLICY_FRESH

    def __init__(self, grids, capacity: int = 64, num_blocks: int | None = None, stream=None,
                 device="cuda", bulk_min: int | None = None, bitmap_width: int = 64):
        self.sides = np.array([g.shape[0] for g in grids], dtype=np.uint32)
        for g in grids:
            assert g.shape[0] == g.shape[1], "worlds are square"
        self.total = int((self.sides.astype(np.int64) ** 2).sum())
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        blocks = num_blocks or gol_blocks_for(self.total, capacity)
        self.heap = Heap(blocks, capacity, GOL_TYPES, device=device, stream=self.stream, bitmap_width=bitmap_width)
        self.heap.set_policy(self.BULK_MIN if bulk_min is None else bulk_min)
        self.heap.set_type_policy(GOL_CAND, self.CAND_POLICY)
        self.lib = self.heap.lib
        nbytes = int(self.lib.dsoar_gol_bytes(len(grids), self.sides.ctypes.data))
        if nbytes == 0:
            raise ValueError("bad world sizes")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        flat = np.concatenate([np.ascontiguousarray(g, dtype=np.uint8).ravel() for g in grids])
        with torch.cuda.stream(self.stream):
            self.grid0 = torch.from_numpy(flat).to(device)
        self.out = torch.empty(self.total, dtype=torch.uint8, device=device)
        g = ctypes.c_void_p()
        C.check(self.lib.dsoar_gol_create(self.heap.h, len(grids), self.sides.ctypes.data, self.buf.data_ptr(),
                                          nbytes, self.heap._s(), ctypes.byref(g)), "dsoar_gol_create")
        self.g = g

    def close(self):
        if getattr(self, "g", None):
            self.lib.dsoar_gol_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self):
        self.heap.reset()
        C.check(self.lib.dsoar_gol_init(self.g, self.grid0.data_ptr(), self.heap._s()), "dsoar_gol_init")

    def step(self, generations: int, flags: int = C.DO_PERSISTENT):
        C.check(self.lib.dsoar_gol_step(self.g, generations, flags, self.heap._s()), "dsoar_gol_step")

    def read(self) -> list:
        C.check(self.lib.dsoar_gol_read(self.g, self.out.data_ptr(), self.heap._s()), "dsoar_gol_read")
        self.stream.synchronize()
        flat = self.out.cpu().numpy()
        grids, off = [], 0
        for s in self.sides.tolist():
            grids.append(flat[off: off + s * s].reshape(s, s))
            off += s * s
        return grids

    def synchronize(self):
        self.stream.synchronize()


# -------------------------------------------------------------- sugarscape --

SUGAR_TYPE = [(4, 4, 4, 4, 4, 4, 4)]  # Agent {sugar, metabolism, vision, age, pos, target, world}


@dataclass
class SugarGpuState:
    side: int
    sugar: np.ndarray
    occ: np.ndarray
    a_sugar: np.ndarray
    a_metab: np.ndarray
    a_vision: np.ndarray
    a_age: np.ndarray
    moves: int
    stats: dict


SUGAR_MAX = 127  # a cell keeps its sugar and capacity in seven bits


class Sugarscape:
    """The Sugarscape-style agent model of one world as objects in a device heap."""

    def __init__(self, inp, rules: dict, capacity: int = 64, num_blocks: int | None = None, stream=None,
                 device="cuda"):
        self.side = inp.side
        n = self.side * self.side
        for name in ("sugar", "cap"):
            a = np.asarray(getattr(inp, name))
            if a.size and (a.min() < 0 or a.max() > SUGAR_MAX):
                raise ValueError(f"{name} per cell must lie in 0..{SUGAR_MAX}")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        blocks = num_blocks or max(64, 1 << (max(1, -(-n // (capacity or 64))) - 1).bit_length())
        self.heap = Heap(blocks, capacity, SUGAR_TYPE, device=device, stream=self.stream)
        self.lib = self.heap.lib
        nbytes = int(self.lib.dsoar_sugar_bytes(self.side))
        if nbytes == 0:
            raise ValueError("bad side")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.rules = C.SugarRules(rules["max_age"], rules["repro_min"], rules["fertile_min"],
                                  rules["fertile_max"], int(inp.seed))
        with torch.cuda.stream(self.stream):
            self.inputs = [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in
                           (inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab, inp.a_vision, inp.a_age)]
            self.out = [torch.empty(n, dtype=dt, device=device) for dt in
                        (torch.int32, torch.uint8, torch.int32, torch.int32, torch.int32, torch.int32)]
        s = ctypes.c_void_p()
        C.check(self.lib.dsoar_sugar_create(self.heap.h, self.side, ctypes.byref(self.rules), self.buf.data_ptr(),
                                            nbytes, ctypes.byref(s)), "dsoar_sugar_create")
        self.s = s

    def close(self):
        if getattr(self, "s", None):
            self.lib.dsoar_sugar_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, step0: int = 0):
        self.heap.reset()
        C.check(self.lib.dsoar_sugar_init(self.s, *[t.data_ptr() for t in self.inputs], step0, self.heap._s()),
                "dsoar_sugar_init")

    def step(self, steps: int, flags: int = C.DO_PERSISTENT):
        C.check(self.lib.dsoar_sugar_step(self.s, steps, flags, self.heap._s()), "dsoar_sugar_step")

    def read(self) -> SugarGpuState:
        moves = ctypes.c_uint32()
        C.check(self.lib.dsoar_sugar_read(self.s, *[t.data_ptr() for t in self.out], ctypes.byref(moves),
                                          self.heap._s()), "dsoar_sugar_read")
        self.stream.synchronize()
        a = [t.cpu().numpy() for t in self.out]
        return SugarGpuState(self.side, a[0], a[1], a[2], a[3], a[4], a[5], int(moves.value),
                             self.heap.stats(raise_sticky=False))

    def synchronize(self):
        self.stream.synchronize()


# ---------------------------------------------------------------- traffic --

TRAFFIC_TYPE = [(4, 4, 4)]  # Car {cell, speed, next speed}


class Traffic:
    """Nagel-Schreckenberg traffic on open roads, Car objects in a device heap."""

    def __init__(self, inp, rules: dict, capacity: int = 64, num_blocks: int | None = None, stream=None,
                 device="cuda"):
        self.roads, self.length = inp.roads, inp.length
        n = self.roads * self.length
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        # At most one car per cell, plus partly filled blocks.
        blocks = num_blocks or max(64, 1 << (2 * -(-n // (capacity or 64)) - 1).bit_length())
        self.heap = Heap(blocks, capacity, TRAFFIC_TYPE, device=device, stream=self.stream)
        # Cars leave their blocks one by one, so the active blocks hold a slot
        # or two each: the entering cars take at most two lookups' worth of
        # them and a free block for the rest (16.9 against 23.1 ms per 500
        # steps of 1024 roads on MI355X, 28 % more blocks, same results).
        self.heap.set_type_policy(0, C.POLICY_BOUNDED)
        self.lib = self.heap.lib
        nbytes = int(self.lib.dsoar_traffic_bytes(self.roads, self.length))
        if nbytes == 0:
            raise ValueError("bad road size")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.rules = C.TrafficRules(rules["vmax"], rules["p_slow24"], rules["p_in24"], 0, int(inp.seed))
        with torch.cuda.stream(self.stream):
            self.vel0 = torch.from_numpy(np.ascontiguousarray(inp.vel, dtype=np.int32).ravel()).to(device)
            self.out = torch.empty(n, dtype=torch.int32, device=device)
        t = ctypes.c_void_p()
        C.check(self.lib.dsoar_traffic_create(self.heap.h, self.roads, self.length, ctypes.byref(self.rules),
                                              self.buf.data_ptr(), nbytes, ctypes.byref(t)), "dsoar_traffic_create")
        self.t = t

    def close(self):
        if getattr(self, "t", None):
            self.lib.dsoar_traffic_destroy(self.t)
            self.t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, step0: int = 0):
        self.heap.reset()
        C.check(self.lib.dsoar_traffic_init(self.t, self.vel0.data_ptr(), step0, self.heap._s()),
                "dsoar_traffic_init")

    def step(self, steps: int, flags: int = C.DO_PERSISTENT):
        C.check(self.lib.dsoar_traffic_step(self.t, steps, flags, self.heap._s()), "dsoar_traffic_step")

    def read(self) -> np.ndarray:
        C.check(self.lib.dsoar_traffic_read(self.t, self.out.data_ptr(), self.heap._s()), "dsoar_traffic_read")
        self.stream.synchronize()
        return self.out.cpu().numpy().reshape(self.roads, self.length)

    def synchronize(self):
        self.stream.synchronize()


# ------------------------------------------------------------- collisions --

BODY_TYPE = [(4,) * 8]  # Body {x, y, vx, vy, ax, ay, m, id}


@dataclass
class CollideGpuState:
    x: np.ndarray
    y: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    m: np.ndarray
    stats: dict


class Collisions:
    """Merging bodies in the plane, Body objects in a device heap."""

    def __init__(self, inp, params: dict, capacity: int = 64, num_blocks: int | None = None, stream=None,
                 device="cuda"):
        self.n = inp.n
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        blocks = num_blocks or max(64, 1 << (2 * -(-self.n // (capacity or 64)) - 1).bit_length())
        self.heap = Heap(blocks, capacity, BODY_TYPE, device=device, stream=self.stream)
        self.lib = self.heap.lib
        nbytes = int(self.lib.dsoar_collide_bytes(self.n))
        if nbytes == 0:
            raise ValueError("bad body count")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.params = C.CollideParams(params["dt"], params["eps2"], params["r2_merge"], 0)
        with torch.cuda.stream(self.stream):
            self.inputs = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
                           for a in (inp.x, inp.y, inp.vx, inp.vy, inp.m)]
            self.out = [torch.empty(self.n, dtype=torch.float32, device=device) for _ in range(5)]
        c = ctypes.c_void_p()
        C.check(self.lib.dsoar_collide_create(self.heap.h, self.n, ctypes.byref(self.params), self.buf.data_ptr(),
                                              nbytes, ctypes.byref(c)), "dsoar_collide_create")
        self.c = c

    def close(self):
        if getattr(self, "c", None):
            self.lib.dsoar_collide_destroy(self.c)
            self.c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self):
        self.heap.reset()
        C.check(self.lib.dsoar_collide_init(self.c, *[t.data_ptr() for t in self.inputs], self.heap._s()),
                "dsoar_collide_init")

    def step(self, steps: int, flags: int = C.DO_PERSISTENT):
        C.check(self.lib.dsoar_collide_step(self.c, steps, flags, self.heap._s()), "dsoar_collide_step")

    def read(self) -> CollideGpuState:
        C.check(self.lib.dsoar_collide_read(self.c, *[t.data_ptr() for t in self.out], self.heap._s()),
                "dsoar_collide_read")
        self.stream.synchronize()
        a = [t.cpu().numpy() for t in self.out]
        return CollideGpuState(*a, stats=self.heap.stats(raise_sticky=False))

    def synchronize(self):
        self.stream.synchronize()


# ------------------------------------------------------------------ wa-tor --

WATOR_TYPES = [(4, 4, 4), (4, 4, 4, 4)]  # Fish {pos, age, target}, Shark {pos, age, energy, target}


@dataclass
class WatorGpuState:
    kind: np.ndarray     # int32 [side, side]
    age: np.ndarray
    energy: np.ndarray
    stats: dict


class Wator:
    """Wa-Tor fish and sharks on a torus, Fish and Shark objects in a device heap."""

    def __init__(self, inp, rules: dict, capacity: int = 64, num_blocks: int | None = None, stream=None,
                 device="cuda"):
        self.side = inp.side
        n = self.side * self.side
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        # At most one animal per cell; room for both types' partly filled blocks.
        blocks = num_blocks or max(64, 1 << (4 * -(-n // (capacity or 64)) - 1).bit_length())
        self.heap = Heap(blocks, capacity, WATOR_TYPES, device=device, stream=self.stream)
        # Fish and sharks leave holes one by one (eaten, starved): their
        # newborns take at most two lookups' worth of holes and a free block
        # for the rest (57.6 against 60.8 ms per 200 steps of 2048^2 on MI355X,
        # 7 % more blocks, same results).
        for t in range(len(WATOR_TYPES)):
            self.heap.set_type_policy(t, C.POLICY_BOUNDED)
        self.lib = self.heap.lib
        nbytes = int(self.lib.dsoar_wator_bytes(self.side))
        if nbytes == 0:
            raise ValueError("bad sea size")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.rules = C.WatorRules(rules["fish_breed"], rules["shark_breed"], rules["starve"], 0, int(inp.seed))
        with torch.cuda.stream(self.stream):
            self.inputs = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32).ravel()).to(device)
                           for a in (inp.kind, inp.age, inp.energy)]
            self.out = [torch.empty(n, dtype=torch.int32, device=device) for _ in range(3)]
        w = ctypes.c_void_p()
        C.check(self.lib.dsoar_wator_create(self.heap.h, self.side, ctypes.byref(self.rules), self.buf.data_ptr(),
                                            nbytes, ctypes.byref(w)), "dsoar_wator_create")
        self.w = w

    def close(self):
        if getattr(self, "w", None):
            self.lib.dsoar_wator_destroy(self.w)
            self.w = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, step0: int = 0):
        self.heap.reset()
        k, a, e = self.inputs
        C.check(self.lib.dsoar_wator_init(self.w, k.data_ptr(), a.data_ptr(), e.data_ptr(), step0, self.heap._s()),
                "dsoar_wator_init")

    def step(self, steps: int, flags: int = C.DO_PERSISTENT):
        C.check(self.lib.dsoar_wator_step(self.w, steps, flags, self.heap._s()), "dsoar_wator_step")

    def read(self) -> WatorGpuState:
        k, a, e = self.out
        C.check(self.lib.dsoar_wator_read(self.w, k.data_ptr(), a.data_ptr(), e.data_ptr(), self.heap._s()),
                "dsoar_wator_read")
        self.stream.synchronize()
        shape = (self.side, self.side)
        return WatorGpuState(k.cpu().numpy().reshape(shape), a.cpu().numpy().reshape(shape),
                             e.cpu().numpy().reshape(shape), self.heap.stats())

    def synchronize(self):
        self.stream.synchronize()
