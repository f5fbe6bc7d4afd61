"""Serving: episodes (Game-of-Life and Sugarscape worlds) arrive over time,
are admitted by free-block budget into two resident world pools, and are
advanced together, one generation / step per server step (continuous
batching: a world joins at the first step boundary after it fits and leaves
at the first boundary after it finishes).  The two pools run on their own
streams, so their kernels overlap on the device.

Every world's evolution depends only on its own state, seed and step count,
so its result is the same whether it runs alone or in the mix."""
from __future__ import annotations

import ctypes
import hashlib
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _capi as C
from .apps import GOL_CAND, GOL_TYPES, SUGAR_TYPE, GameOfLife
from .heap import Heap


def result_digest(kind: str, res) -> str:
    """SHA-256 of an episode's retired state (for comparing runs of the same
    episode without keeping its arrays): the grid of a Game-of-Life world;
    the sugar grid, occupancy, per-cell agent fields and move count of a
    Sugarscape world."""
    h = hashlib.sha256(kind.encode())
    if kind == "gol":
        h.update(np.ascontiguousarray(res, dtype=np.uint8).tobytes())
    else:
        for k in ("sugar", "occ", "a_sugar", "a_metab", "a_vision", "a_age"):
            h.update(np.ascontiguousarray(res[k]).tobytes())
        h.update(str(res["moves"]).encode())
    return h.hexdigest()


class RangeAllocator:
    """First-fit allocator of cell ranges in an arena (host side)."""

    def __init__(self, size: int):
        self.free = [(0, size)]

    def alloc(self, n: int):
        for i, (s, l) in enumerate(self.free):
            if l >= n:
                if l == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + n, l - n)
                return s
        return None

    def release(self, start: int, n: int):
        self.free.append((start, n))
        self.free.sort()
        merged = []
        for s, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((s, l))
        self.free = merged


@dataclass
class Running:
    spec: object
    slot: int
    offset: int
    need: int
    admitted_at: float
    steps: int = 0
    inputs: list = field(default_factory=list)


def gol_need(side: int, capacity: int = 64) -> int:
    # Cells, plus at most one Alive or Candidate per cell, plus partial blocks.
    return 3 * -(-side * side // capacity)


def sugar_need(side: int, capacity: int = 64) -> int:
    # At most one agent per cell.
    return 2 * -(-side * side // capacity)


class Pool:
    """One world pool (GoL or Sugarscape) with its heap, stream and budget."""

    def __init__(self, kind: str, blocks: int, slots: int, arena: int, rules: dict | None = None,
                 graph: bool = True, device="cuda"):
        self.kind = kind
        self.stream = torch.cuda.Stream(device=device)
        types = GOL_TYPES if kind == "gol" else SUGAR_TYPE
        self.heap = Heap(blocks, 64, types, device=device, stream=self.stream)
        if kind == "gol":
            self.heap.set_policy(GameOfLife.BULK_MIN)  # as the single-pool GoL driver
            self.heap.set_type_policy(GOL_CAND, GameOfLife.CAND_POLICY)
        self.lib = self.heap.lib
        self.blocks = blocks
        self.budget = blocks
        self.arena = RangeAllocator(arena)
        self.free_slots = list(range(slots))[::-1]
        self.flags = C.DO_PERSISTENT | (C.GRAPH if graph else 0)
        p = ctypes.c_void_p()
        s = self.heap._s()
        if kind == "gol":
            nbytes = int(self.lib.dsoar_golpool_bytes(slots, arena))
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
            C.check(self.lib.dsoar_golpool_create(self.heap.h, slots, arena, self.buf.data_ptr(), nbytes, s,
                                                  ctypes.byref(p)), "dsoar_golpool_create")
        else:
            nbytes = int(self.lib.dsoar_sugarpool_bytes(slots, arena))
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
            self.rules = C.SugarRules(rules["max_age"], rules["repro_min"], rules["fertile_min"],
                                      rules["fertile_max"], 0)
            C.check(self.lib.dsoar_sugarpool_create(self.heap.h, slots, arena, ctypes.byref(self.rules),
                                                    self.buf.data_ptr(), nbytes, ctypes.byref(p)),
                    "dsoar_sugarpool_create")
        self.p = p
        self.resident: dict[int, Running] = {}

    def need(self, spec) -> int:
        return gol_need(spec.side) if self.kind == "gol" else sugar_need(spec.side)

    def try_admit(self, spec, inputs, now: float) -> bool:
        need = self.need(spec)
        if need > self.budget or not self.free_slots:
            return False
        n = spec.side * spec.side
        off = self.arena.alloc(n)
        if off is None:
            return False
        slot = self.free_slots.pop()
        s = self.heap._s()
        with torch.cuda.stream(self.stream):
            if self.kind == "gol":
                dev = [torch.from_numpy(np.ascontiguousarray(inputs, dtype=np.uint8).ravel()).to("cuda",
                                                                                                 non_blocking=False)]
                C.check(self.lib.dsoar_gol_admit(self.p, slot, off, spec.side, dev[0].data_ptr(), s),
                        "dsoar_gol_admit")
            else:
                dev = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in
                       (inputs.sugar, inputs.cap, inputs.occ, inputs.a_sugar, inputs.a_metab, inputs.a_vision,
                        inputs.a_age)]
                C.check(self.lib.dsoar_sugar_admit(self.p, slot, off, spec.side, spec.seed, 0,
                                                   *[t.data_ptr() for t in dev], s), "dsoar_sugar_admit")
        self.budget -= need
        self.resident[spec.eid] = Running(spec, slot, off, need, now, inputs=dev)
        return True

    def step(self):
        if not self.resident:
            return
        s = self.heap._s()
        if self.kind == "gol":
            C.check(self.lib.dsoar_gol_step(self.p, 1, self.flags, s), "dsoar_gol_step")
        else:
            C.check(self.lib.dsoar_sugar_step(self.p, 1, self.flags, s), "dsoar_sugar_step")
        for r in self.resident.values():
            r.steps += 1
            r.inputs = []  # the admission copies have been consumed

    def finished(self):
        return [r for r in self.resident.values() if r.steps >= r.spec.length]

    def retire(self, r: Running):
        """Reads the world's result, deletes its objects and frees its slot."""
        s = self.heap._s()
        n = r.spec.side * r.spec.side
        with torch.cuda.stream(self.stream):
            if self.kind == "gol":
                out = torch.empty(n, dtype=torch.uint8, device="cuda")
                C.check(self.lib.dsoar_gol_read_world(self.p, r.slot, out.data_ptr(), s), "dsoar_gol_read_world")
                self.stream.synchronize()
                result = out.cpu().numpy().reshape(r.spec.side, r.spec.side)
                C.check(self.lib.dsoar_gol_retire(self.p, r.slot, s), "dsoar_gol_retire")
            else:
                outs = [torch.empty(n, dtype=dt, device="cuda") for dt in
                        (torch.int32, torch.uint8, torch.int32, torch.int32, torch.int32, torch.int32)]
                moves = ctypes.c_uint64()
                C.check(self.lib.dsoar_sugar_read_world(self.p, r.slot, *[t.data_ptr() for t in outs],
                                                        ctypes.byref(moves), s), "dsoar_sugar_read_world")
                result = {k: t.cpu().numpy() for k, t in
                          zip(("sugar", "occ", "a_sugar", "a_metab", "a_vision", "a_age"), outs)}
                result["moves"] = int(moves.value)
                C.check(self.lib.dsoar_sugar_retire(self.p, r.slot, s), "dsoar_sugar_retire")
        self.arena.release(r.offset, n)
        self.free_slots.append(r.slot)
        self.budget += r.need
        del self.resident[r.spec.eid]
        return result

    def close(self):
        if getattr(self, "p", None):
            if self.kind == "gol":
                self.lib.dsoar_gol_destroy(self.p)
            else:
                self.lib.dsoar_sugar_destroy(self.p)
            self.p = None


@dataclass
class Record:
    eid: int
    kind: str
    side: int
    length: int
    arrival: float
    admitted: float
    done: float

    @property
    def latency(self):
        return self.done - self.arrival


class Server:
    """Admits arriving episodes (FIFO, by free-block budget) into the GoL and
    Sugarscape pools and steps all resident worlds together."""

    def __init__(self, gol_blocks=1 << 21, gol_slots=256, gol_arena=1 << 25, sugar_blocks=1 << 19,
                 sugar_slots=64, sugar_arena=1 << 23, rules=None, graph=True, device="cuda"):
        from synth import workloads as W
        self.rules = rules or W.SUGAR_RULES
        self.pools = {"gol": Pool("gol", gol_blocks, gol_slots, gol_arena, graph=graph, device=device),
                      "sugar": Pool("sugar", sugar_blocks, sugar_slots, sugar_arena, self.rules, graph, device)}

    def close(self):
        for p in self.pools.values():
            p.close()

    def fits_ever(self, spec) -> bool:
        p = self.pools[spec.kind]
        return p.need(spec) <= p.blocks

    def check(self) -> dict:
        """Invariant check of both pools' heaps at quiescence (sticky
        out-of-memory, retry-limit and double-free flags included): {} when
        everything holds, else the findings by pool."""
        out = {}
        for name, p in self.pools.items():
            p.stream.synchronize()
            c = p.heap.check()
            if c:
                out[name] = c
        return out

    def run(self, specs, inputs_of, keep_results: bool = True, max_wall: float = 600.0, digests: bool = False):
        """Runs the episodes to completion.  `inputs_of(spec)` returns a
        world's initial state.  Arrival times are seconds after the start on
        the host clock.  Returns (records, results by episode id, stats); with
        digests=True the results are result_digest() strings."""
        queue = sorted(specs, key=lambda e: (e.arrival, e.eid))
        for e in queue:
            if not self.fits_ever(e):
                raise ValueError(f"episode {e.eid} can never fit its pool")
        records, results = [], {}
        qi = 0
        steps = 0
        busy = 0.0
        t0 = time.perf_counter()
        while qi < len(queue) or any(p.resident for p in self.pools.values()):
            now = time.perf_counter() - t0
            if now > max_wall:
                raise TimeoutError("serving run exceeded its wall-clock limit")
            # 1. retire the worlds that finished at the last boundary
            for p in self.pools.values():
                for r in p.finished():
                    res = p.retire(r)
                    done = time.perf_counter() - t0
                    records.append(Record(r.spec.eid, r.spec.kind, r.spec.side, r.spec.length, r.spec.arrival,
                                          r.admitted_at, done))
                    if digests:
                        results[r.spec.eid] = result_digest(r.spec.kind, res)
                    elif keep_results:
                        results[r.spec.eid] = res
            # 2. admit arrived episodes in order while they fit
            now = time.perf_counter() - t0
            while qi < len(queue) and queue[qi].arrival <= now:
                spec = queue[qi]
                if not self.pools[spec.kind].try_admit(spec, inputs_of(spec), now):
                    break  # FIFO: wait for space
                qi += 1
            if not any(p.resident for p in self.pools.values()):
                if qi < len(queue):
                    time.sleep(max(0.0, min(queue[qi].arrival - (time.perf_counter() - t0), 0.01)))
                continue
            # 3. one step of every resident world; the pools overlap on the device
            ts = time.perf_counter()
            for p in self.pools.values():
                p.step()
            for p in self.pools.values():
                p.stream.synchronize()
            busy += time.perf_counter() - ts
            steps += 1
        wall = time.perf_counter() - t0
        return records, results, {"wall_s": wall, "server_steps": steps, "step_busy_s": busy}


def summarize(records, wall: float) -> dict:
    lat = np.array([r.latency for r in records]) if records else np.zeros(1)
    cells_gens = sum(r.side * r.side * r.length for r in records)
    return {"episodes": len(records), "episodes_per_s": len(records) / wall if wall > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()), "cell_steps_per_s": cells_gens / wall if wall > 0 else 0.0}
