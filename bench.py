"""Benchmark of the object heap + parallel do-all on one MI355X.

Default workload: 256 independent Game-of-Life worlds as objects in one heap,
sides log-uniform from 64 to 1024 (48.8 M cells), Bernoulli(0.1) alive, 100
generations.  One step = reset the heap, create every world's initial objects
and run the 100 generations (one persistent do-all per phase covering all
worlds, replayed from HIP graphs), with the seeded input grids already
resident in device memory; block capacity, do-all launch shape and allocation
policy come from the autotuner's cached choice.  The same worlds, each with
its own heap and its own launches one world after another (the plain
baseline), are timed beside it.

Prints one JSON line with the headline throughput (allocations + frees per
second), do-all objects per second, cells x generations per second, the
roofline entry of the dominant kernel (per-launch HIP-event timing over a
profiled pass of the same workload), batched against plain, and the CPU
baseline (the oracle, single thread, on a bounded sample).  --workload
selects the other configurations.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "allocs+frees/sec and do-all objects/sec (HBM GB/s % peak); batched vs plain"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="batched",
                   choices=["gol", "micro", "micro_scaled", "batched", "sugarscape", "traffic", "collisions", "nbody",
                            "wator",
                            "serve"])
    p.add_argument("--episodes", type=int, default=200, help="serve: episodes per arrival rate")
    p.add_argument("--rates", default="0.25,0.5,0.75,0.9,1.1",
                   help="serve: arrival rates as fractions of the measured capacity")
    p.add_argument("--tune", default="cache", choices=["cache", "full", "off"],
                   help="batched: autotune (cached in paper_1809_07444_amd/tune_cache.json), full re-tune, or defaults")
    p.add_argument("--no-plain", action="store_true", help="batched: skip the per-world plain baseline")
    p.add_argument("--seed", type=int, default=24301)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-graph", action="store_true")
    p.add_argument("--traffic-probe", action="store_true",
                   help="after the run, launch one elementwise kernel over 256 MiB (counter calibration)")
    p.add_argument("--scaled-blocks", type=int, default=1 << 22)
    p.add_argument("--probe", action="store_true", help="also measure atomic and copy ceilings")
    p.add_argument("--bulk-min", type=lambda v: 0xFFFFFFFF if v == "never" else int(v), default=None,
                   help="allocation policy: requests of at least this many take whole free blocks first "
                        "('never' = the dense default)")
    p.add_argument("--unroll", type=int, default=None, help="blocks per wavefront pass of split do-alls")
    p.add_argument("--reclaim", default="quiescent", choices=["quiescent", "online"],
                   help="free emptied blocks at enumeration (default) or at the delete that empties them")
    p.add_argument("--bodies", type=int, default=65536,
                   help="collisions: number of bodies (the box side grows with sqrt(bodies), fixed density)")
    return p.parse_args()


# ------------------------------------------------------------- bytes model --
# Algorithmic bytes each kernel kind must move, from the heap's counters over
# the profiled pass.  A do-all visit counts the visited object's own fields
# read and written; an allocation the fields of the object it creates; each
# listed block its entry (4 B id + 8 B snapshot).  Reads and writes of other
# objects' state (a Game of Life cell's neighbours, the Cell a dying or born
# cell updates, the world table) are counted apart as "other" bytes and are
# not part of the roofline's achieved figure.  Kinds may return one number
# (no other-object traffic) or a pair (algorithmic, other).

def gol_kernel_bytes(kind, launches, st, M, init_alive):
    A, K = 1, 2  # Alive, Candidate type ids
    va, vk = st["visits"][A] / 2, st["visits"][K] / 2     # each type is visited by two do-alls
    cands = st["allocs"][K]
    births, deaths = st["allocs"][A] - init_alive, st["frees"][A]
    if kind == "gol_alive_prep":
        # this: cell and world read, action written; new Candidates: their
        # three fields; other: the live bits of the 24 surrounding cells and
        # the world's offset and side.
        return va * 12 + cands * 12 + va / 64 * 12, va * (3 + 8)
    if kind == "gol_cand_prep":
        return vk * 12 + vk / 64 * 12, vk * (1 + 8)
    if kind == "gol_alive_update":
        # this: action read, and the cell of a dying one; other: its Cell's
        # index word and field and its live byte.
        return va * 4 + deaths * 4 + va / 64 * 12, deaths * (4 + 4 + 1)
    if kind == "gol_cand_update":
        # this: cell, world and action read; new Alive objects: three fields;
        # other: the born cell's index word, Cell field and live byte.
        return vk * 12 + births * 12 + vk / 64 * 12, births * (4 + 4 + 1)
    if kind == "gol_update":  # phases 3 and 4 in one launch
        a = gol_kernel_bytes("gol_alive_update", launches, st, M, init_alive)
        c = gol_kernel_bytes("gol_cand_update", launches, st, M, init_alive)
        return a[0] + c[0], a[1] + c[1]
    if kind == "enumerate":
        return launches * (M / 8) + (va + vk) / 64 * 20
    return None


def gol_init_bytes(cells, alive):
    # New objects: each Cell's field, each initial Alive's three fields.
    # Other: the input byte, the index word and live byte of every cell.
    return cells * 4 + alive * 12 + (cells + alive) / 64 * 12, cells * (1 + 4 + 1)


def sugar_kernel_bytes(kind, launches, st, M, init_agents, cells):
    """(this + new-object bytes, other bytes) of the Sugarscape kernels.  Per
    agent visit, this: choose reads pos, vision and world and writes target;
    move reads pos, target and world and writes pos; eat reads pos, sugar,
    metabolism and age and writes sugar and age; request reads sugar and age
    and writes target; birth reads target, pos and world.  New objects: a
    child's seven fields.  Other: the grid cells in sight (one byte each, 25
    loaded), the world table, request words and the cells a move, meal,
    request or birth touches."""
    v = st["visits"][0] / 5  # five do-alls per step
    births = st["allocs"][0] - init_agents
    per = {"sugar_choose": (16, 25 + 8 + 4), "sugar_move": (16, 4 + 16), "sugar_eat": (24, 2 + 4),
           "sugar_request": (12, 8 + 16 + 4), "sugar_birth": (12, 4)}
    if kind in per:
        this, other = per[kind]
        if kind == "sugar_birth":  # a child's seven fields; its cell's occupant word and byte
            return v * this + v / 64 * 12 + births * 28, v * other + births * 5
        return v * this + v / 64 * 12, v * other
    if kind == "sugar_regrow":  # other state only: sugar byte and capacity read, sugar byte written, per cell
        return 0.0, launches * cells * 6
    if kind == "enumerate":
        return launches * (M / 8) + (2 * v / 64) * 20
    return None


def micro_kernel_bytes(kind, launches, st, M):
    v = st["visits"][0] / 2  # update and cull visit the same objects
    if kind == "micro_update":
        return v * 12 + v / 64 * 12
    if kind == "micro_cull":
        return v * 4 + st["frees"][0] * 0 + v / 64 * 12 + v / 64 * 8
    if kind == "micro_create":
        # x and v read from the inputs, id, x and v written; per block taken
        # its object bitmap and type word.
        return st["allocs"][0] * 20 + st["allocs"][0] / 64 * 12
    if kind == "enumerate":
        return launches * (M / 8) + v / 64 * 20
    return None


# --------------------------------------------------------------- workloads --

class GolWorkload:
    name = "gol"

    def __init__(self, args):
        import torch
        from paper_1809_07444_amd import _capi as C
        from paper_1809_07444_amd import apps
        from synth import workloads as W
        self.C = C
        self.side, self.gens = 1024, 200
        self.grid = W.gol_grid(self.side, self.side, seed=args.seed)
        self.gol = apps.GameOfLife([self.grid])
        self.init_objects = (int(self.grid.size), int((self.grid != 0).sum()))
        self.flags = C.DO_PERSISTENT | (0 if args.no_graph else C.GOL_GRAPH)
        self.M = self.gol.heap.num_blocks
        self.stream = self.gol.stream
        self.torch = torch
        self.cells_gens = self.side ** 2 * self.gens
        self.config = {"workload": f"gol-{self.side}x{self.side}-bernoulli0.1-{self.gens}gen",
                       "worlds": 1, "cells": self.side ** 2, "generations": self.gens,
                       "heap_blocks": self.M, "block_capacity": 64, "graph": not args.no_graph,
                       "seed": args.seed}

    def step(self):
        self.gol.init()
        self.gol.step(self.gens, self.flags)

    def profiled_step(self):
        # Same work, eager persistent launches, so each kernel is bracketed by events.
        self.gol.init()
        self.gol.step(self.gens, self.C.DO_PERSISTENT)

    def stats(self):
        return self.gol.heap.stats()

    def kernel_bytes(self, kind, launches, st):
        if kind == "gol_init":
            return gol_init_bytes(*self.init_objects)
        return gol_kernel_bytes(kind, launches, st, self.M, self.init_objects[1])

    def heap(self):
        return self.gol.heap

    def cpu_baseline(self):
        import oracle
        t0 = time.perf_counter()
        oracle.gol_run(self.grid, self.gens)
        dt = time.perf_counter() - t0
        # The oracle is a dense stencil: it updates every cell of every
        # generation and allocates nothing, so its rate is cells x generations
        # per second (compare with the line's cells_gens_per_s).
        return {"value": self.side ** 2 * self.gens / dt, "unit": "cells*gens/s", "cores": 1, "kind": "oracle",
                "sample": f"dense B3/S23 oracle, full {self.side}x{self.side} torus, {self.gens} generations, "
                          f"{dt:.2f} s"}


class MicroWorkload:
    name = "micro"

    def __init__(self, args, scaled=False):
        import torch
        from paper_1809_07444_amd import _capi as C
        from paper_1809_07444_amd import apps
        from synth import workloads as W
        self.C = C
        if scaled:
            self.name = "micro_scaled"
            self.M = args.scaled_blocks
            n, steps = 16 * self.M, 2
        else:
            self.M, n, steps = 4096, 65536, 10
        self.inp = W.micro_inputs(n, steps, seed=args.seed)
        self.mb = apps.MicroBench(self.inp, self.M, 64)
        self.torch = torch
        self.stream = None
        self.config = {"workload": f"micro-{n}obj-{self.M}blocks-{steps}steps" + ("-scaled" if scaled else ""),
                       "objects": n, "heap_blocks": self.M, "block_capacity": 64, "steps": steps,
                       "seed": args.seed}

    def step(self):
        self.mb.run()

    profiled_step = step

    def stats(self):
        return self.mb.heap.stats()

    def kernel_bytes(self, kind, launches, st):
        return micro_kernel_bytes(kind, launches, st, self.M)

    def heap(self):
        return self.mb.heap

    def cpu_baseline(self):
        import oracle
        from synth import workloads as W
        n = min(self.inp.n_init, 1 << 22)
        inp = self.inp if n == self.inp.n_init else W.micro_inputs(n, self.inp.steps)
        t0 = time.perf_counter()
        r = oracle.micro_run(inp)
        dt = time.perf_counter() - t0
        return {"value": (r.allocs + r.frees) / dt, "unit": "allocs+frees/s", "cores": 1, "kind": "oracle",
                "sample": f"micro oracle, {n} objects x {inp.steps} steps, {dt:.3f} s"}


class BatchedWorkload(GolWorkload):
    name = "batched"

    def __init__(self, args):
        import torch
        from paper_1809_07444_amd import _capi as C
        from paper_1809_07444_amd import batch
        from synth import workloads as W
        self.C, self.batch, self.torch = C, batch, torch
        self.gens = 100
        self.inp = W.batch_inputs(256, self.gens, seed=args.seed)
        cache = os.path.join(ROOT, "paper_1809_07444_amd", "tune_cache.json")
        self.tune_table = None
        if args.tune == "off":
            cfg = batch.TuneConfig()
        else:
            if args.tune == "full" and os.path.exists(cache):
                os.remove(cache)
            log = lambda m: print(m, file=sys.stderr, flush=True)
            cfg, self.tune_table = batch.autotune(self.inp.grids, 10, cache_path=cache, log=log)
        self.cfg = cfg
        self.b = batch.BatchedGol(self.inp.grids, cfg)
        self.init_objects = (sum(int(g.size) for g in self.inp.grids),
                             sum(int((g != 0).sum()) for g in self.inp.grids))
        self.gol = self.b.gol
        self.M = self.gol.heap.num_blocks
        self.cells_gens = int(self.gol.total) * self.gens
        self.args = args
        from dataclasses import asdict
        self.config = {"workload": f"gol-batched-256worlds-loguniform64..1024-bernoulli0.1-{self.gens}gen",
                       "worlds": 256, "cells": int(self.gol.total), "generations": self.gens,
                       "heap_blocks": self.M, "tuned": asdict(cfg), "graph": True, "seed": args.seed}

    def step(self):
        self.b.run(self.gens)

    def profiled_step(self):
        self.gol.init()
        self.gol.step(self.gens, self.C.DO_PERSISTENT)

    def plain_baseline(self):
        import torch
        out = {}
        for name, sync in (("plain", False), ("plain_sync", True)):
            p = self.batch.PlainGol(self.inp.grids, capacity=64, sync=sync)
            p.run(1)
            p.synchronize()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.run(self.gens)
            p.synchronize()
            out[name + "_ms"] = (time.perf_counter() - t0) * 1e3
            del p
            torch.cuda.empty_cache()
        return out

    def cpu_baseline(self):
        import oracle
        # Bounded sample: the first worlds in order until ~10 s of oracle work.
        # The oracle is a dense stencil (no allocation): cells x generations per second.
        t0 = time.perf_counter()
        cells = 0
        n = 0
        for g in self.inp.grids:
            oracle.gol_run(g, self.gens)
            cells += g.size
            n += 1
            if time.perf_counter() - t0 > 10:
                break
        dt = time.perf_counter() - t0
        return {"value": cells * self.gens / dt, "unit": "cells*gens/s", "cores": 1, "kind": "oracle",
                "sample": f"dense B3/S23 oracle on the first {n} of 256 worlds ({cells} cells), {self.gens} "
                          f"generations, {dt:.1f} s"}


class SugarWorkload(GolWorkload):
    name = "sugarscape"

    def __init__(self, args):
        import torch
        from paper_1809_07444_amd import _capi as C
        from paper_1809_07444_amd import apps
        from synth import workloads as W
        self.C, self.torch = C, torch
        self.side, self.agents, self.steps = 2048, 1 << 20, 500
        self.inp = W.sugar_inputs(self.side, self.agents, seed=args.seed)
        self.sim = apps.Sugarscape(self.inp, W.SUGAR_RULES)
        self.flags = C.DO_PERSISTENT | (0 if args.no_graph else C.GRAPH)
        self.M = self.sim.heap.num_blocks
        self.config = {"workload": f"sugarscape-{self.side}x{self.side}-{self.agents}agents-{self.steps}steps",
                       "cells": self.side ** 2, "agents": self.agents, "steps": self.steps,
                       "heap_blocks": self.M, "block_capacity": 64, "graph": not args.no_graph, "seed": args.seed,
                       "rules": W.SUGAR_RULES}

    def step(self):
        self.sim.init()
        self.sim.step(self.steps, self.flags)

    def profiled_step(self):
        self.sim.init()
        self.sim.step(self.steps, self.C.DO_PERSISTENT)

    def stats(self):
        return self.sim.heap.stats()

    def heap(self):
        return self.sim.heap

    def kernel_bytes(self, kind, launches, st):
        return sugar_kernel_bytes(kind, launches, st, self.M, self.agents, self.side ** 2)

    def cpu_baseline(self):
        import oracle
        from synth import workloads as W
        st = oracle.SugarState(self.side, self.inp.sugar, self.inp.cap, self.inp.occ, self.inp.a_sugar,
                               self.inp.a_metab, self.inp.a_vision, self.inp.a_age)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < 10 and n < self.steps:
            st = oracle.sugar_run(st, 5, self.inp.seed, W.SUGAR_RULES, step0=n)
            n += 5
        dt = time.perf_counter() - t0
        ops = st.births + st.deaths
        return {"value": ops / dt, "unit": "allocs+frees/s", "cores": 1, "kind": "oracle",
                "sample": f"sequential rules oracle, full {self.side}x{self.side} world, first {n} of "
                          f"{self.steps} steps, {dt:.1f} s; births+deaths / oracle time"}


class TrafficWorkload(GolWorkload):
    name = "traffic"

    def __init__(self, args):
        import torch
        from paper_1809_07444_amd import _capi as C
        from paper_1809_07444_amd import apps
        from synth import workloads as W
        self.C, self.torch = C, torch
        self.roads, self.length, self.steps = 1024, 1024, 500
        self.inp = W.traffic_inputs(self.roads, self.length, seed=args.seed)
        self.rules = W.TRAFFIC_RULES
        self.sim = apps.Traffic(self.inp, self.rules)
        self.flags = C.DO_PERSISTENT | (0 if args.no_graph else C.GRAPH)
        self.M = self.sim.heap.num_blocks
        self.config = {"workload": f"traffic-{self.roads}roads-{self.length}cells-density0.15-{self.steps}steps",
                       "roads": self.roads, "cells": self.roads * self.length, "steps": self.steps,
                       "heap_blocks": self.M, "block_capacity": 64, "graph": not args.no_graph, "seed": args.seed,
                       "rules": self.rules}

    def step(self):
        self.sim.init()
        self.sim.step(self.steps, self.flags)

    def profiled_step(self):
        self.sim.init()
        self.sim.step(self.steps, self.C.DO_PERSISTENT)

    def stats(self):
        return self.sim.heap.stats()

    def heap(self):
        return self.sim.heap

    def kernel_bytes(self, kind, launches, st):
        v = st["visits"][0] / 2  # two do-alls per step visit every car
        # (this + new objects, other).  Decide: cell and speed read, next
        # speed written; other: up to vmax road cells ahead.  Drive: next
        # speed and cell read, speed and cell written; other: two road cells.
        per = {"traffic_decide": (12, 4 * self.rules["vmax"]), "traffic_drive": (16, 8)}
        if kind in per:
            return v * per[kind][0] + v / 64 * 12, v * per[kind][1]
        cars0 = int((self.inp.vel >= 0).sum())
        if kind == "traffic_entry":
            # new cars: three fields each; other: every road's first cell read
            # and an entering car's first cell written
            entered = st["allocs"][0] - cars0
            return entered * 12, launches * self.roads * 4 + entered * 4
        if kind == "traffic_init":  # new cars' fields; other: input speed read and cell written per cell
            return cars0 * 12 + cars0 / 64 * 12, self.roads * self.length * 8
        if kind == "enumerate":
            return launches * (self.M / 8) + v / 64 * 20
        return None

    def cpu_baseline(self):
        import oracle
        t0 = time.perf_counter()
        r = oracle.traffic_run(self.inp.vel, self.steps, self.inp.seed, self.rules)
        dt = time.perf_counter() - t0
        ops = int((self.inp.vel >= 0).sum()) + r.entries + r.exits
        return {"value": ops / dt, "unit": "allocs+frees/s", "cores": 1, "kind": "oracle",
                "sample": f"sequential Nagel-Schreckenberg oracle, full {self.roads}x{self.length} roads, "
                          f"{self.steps} steps, {dt:.2f} s; initial cars + entries + exits / oracle time"}


class WatorWorkload(GolWorkload):
    name = "wator"

    def __init__(self, args):
        import torch
        from paper_1809_07444_amd import _capi as C
        from paper_1809_07444_amd import apps
        from synth import workloads as W
        self.C, self.torch = C, torch
        self.side, self.steps = 2048, 200
        self.inp = W.wator_inputs(self.side, seed=args.seed)
        self.rules = W.WATOR_RULES
        self.sim = apps.Wator(self.inp, self.rules)
        self.flags = C.DO_PERSISTENT | (0 if args.no_graph else C.GRAPH)
        self.M = self.sim.heap.num_blocks
        self.config = {"workload": f"wator-{self.side}x{self.side}-fish0.30-sharks0.05-{self.steps}steps",
                       "cells": self.side * self.side, "steps": self.steps, "heap_blocks": self.M,
                       "block_capacity": 64, "graph": not args.no_graph, "seed": args.seed, "rules": self.rules}

    def step(self):
        self.sim.init()
        self.sim.step(self.steps, self.flags)

    def profiled_step(self):
        self.sim.init()
        self.sim.step(self.steps, self.C.DO_PERSISTENT)

    def stats(self):
        return self.sim.heap.stats()

    def heap(self):
        return self.sim.heap

    def kernel_bytes(self, kind, launches, st):
        vf, vs = st["visits"][0] / 3, st["visits"][1] / 2  # three fish do-alls, two shark do-alls per step
        # Fields read and written, the four neighbours' kinds, the request
        # word (an atomic in Decide, a read in Move), the sea cells written,
        # and the newborns' fields.
        # (this, other) per visit: the animal's own fields; the four
        # neighbours' kinds, the request words and the sea cells written.
        per_f = {"wator_fish_decide": (8, 16 + 8), "wator_fish_move": (12, 8 + 16), "wator_fish_eaten": (8, 0)}
        per_s = {"wator_shark_decide": (12, 16 + 8), "wator_shark_move": (16, 12 + 20)}
        fish0 = int((self.inp.kind == 1).sum())
        shark0 = int((self.inp.kind == 2).sum())
        if kind in per_f:
            born = (st["allocs"][0] - fish0) * 12 if kind == "wator_fish_move" else 0  # newborns' fields
            return vf * per_f[kind][0] + vf / 64 * 12 + born, vf * per_f[kind][1]
        if kind in per_s:
            born = (st["allocs"][1] - shark0) * 16 if kind == "wator_shark_move" else 0
            return vs * per_s[kind][0] + vs / 64 * 12 + born, vs * per_s[kind][1]
        if kind == "wator_init":
            # new animals' fields; other: kind, age, energy read, sea byte
            # and request word written per cell
            return fish0 * 12 + shark0 * 16 + (fish0 + shark0) / 64 * 12, self.side ** 2 * (12 + 1 + 8)
        if kind == "wator_tick":
            return launches * 8
        if kind == "enumerate":
            return launches * (self.M / 8) + (vf + vs) / 64 * 20
        return None

    def cpu_baseline(self):
        import oracle
        st = oracle.WatorState(self.inp.kind, self.inp.age, self.inp.energy)
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < 10 and k < self.steps:
            st = oracle.wator_run(st, 1, self.inp.seed, self.rules, step0=k)
            k += 1
        dt = time.perf_counter() - t0
        ops = int((self.inp.kind > 0).sum()) * k / self.steps + st.fish_born + st.sharks_born + \
            st.fish_eaten + st.sharks_starved
        return {"value": ops / dt, "unit": "allocs+frees/s", "cores": 1, "kind": "oracle",
                "sample": f"sequential Wa-Tor oracle, full {self.side}x{self.side} sea, first {k} of {self.steps} "
                          f"steps, {dt:.1f} s; births + meals + starvations (+ the initial animals pro rata) "
                          f"/ oracle time"}


class CollideWorkload(GolWorkload):
    name = "collisions"
    # Per body pair in the force do-all: 2 subtractions, 2 fma (4 flops) for
    # r2, square root, multiplication, division, 2 fma (4 flops) = 13.
    FLOPS_PER_PAIR = 13

    def __init__(self, args):
        import torch
        from paper_1809_07444_amd import _capi as C
        from paper_1809_07444_amd import apps
        from synth import workloads as W
        self.C, self.torch = C, torch
        # 16384 bodies in a 16 x 16 box; other counts keep that density.
        self.n, self.steps = args.bodies, 20
        self.box = float(16.0 * math.sqrt(self.n / 16384))
        self.inp = W.collide_inputs(self.n, seed=args.seed, box=self.box)
        self.params = dict(W.COLLIDE_PARAMS, r2_merge=0.0) if args.workload == "nbody" else W.COLLIDE_PARAMS
        self.doalls = 6  # do-alls per step, each visiting every live body
        if args.workload == "nbody":
            self.name = "nbody"  # merge radius 0: force and move only
            self.doalls = 2
        self.sim = apps.Collisions(self.inp, self.params)
        self.flags = C.DO_PERSISTENT | (0 if args.no_graph else C.GRAPH)
        self.M = self.sim.heap.num_blocks
        self.config = {"workload": f"{self.name}-{self.n}bodies-box{self.box:g}-{self.steps}steps",
                       "bodies": self.n, "steps": self.steps, "heap_blocks": self.M, "block_capacity": 64,
                       "graph": not args.no_graph, "seed": args.seed, "params": self.params}

    def step(self):
        self.sim.init()
        self.sim.step(self.steps, self.flags)

    def profiled_step(self):
        self.sim.init()
        self.sim.step(self.steps, self.C.DO_PERSISTENT)

    def stats(self):
        return self.sim.heap.stats()

    def heap(self):
        return self.sim.heap

    def kernel_flops(self, kind, launches, st):
        if kind != "collide_force":
            return None
        v = st["visits"][0] / self.doalls
        return v * self.n * self.FLOPS_PER_PAIR

    def kernel_bytes(self, kind, launches, st):
        v = st["visits"][0] / self.doalls
        per = {"collide_force": 12 + 8 + 16 * 0, "collide_move": 32 + 24, "collide_root": 12 + 4,
               "collide_target": 16 + 4, "collide_merge": 24 + 4, "collide_remove": 8}
        if kind in per:
            return v * per[kind] + v / 64 * 12
        if kind == "collide_init":
            # five input arrays read; the per-id arrays (16 + 8 + 4 B) and the
            # eight fields of every body written
            return self.n * (20 + 28 + 32) + self.n / 64 * 12
        if kind == "enumerate":
            return launches * (self.M / 8) + v / 64 * 20
        return None

    def cpu_baseline(self):
        import oracle
        st = oracle.CollideState(self.inp.x, self.inp.y, self.inp.vx, self.inp.vy, self.inp.m)
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < 10 and k < self.steps:
            st = oracle.collide_run(st, 1, self.params)
            k += 1
        dt = time.perf_counter() - t0
        pairs = self.n * self.n * k
        ops = int((self.inp.m > 0).sum()) + st.merges
        return {"value": ops / dt, "unit": "allocs+frees/s", "cores": 1, "kind": "oracle",
                "force_tflops": pairs * self.FLOPS_PER_PAIR / dt / 1e12,
                "sample": f"sequential {self.name} oracle, all {self.n} bodies, first {k} of {self.steps} steps, "
                          f"{dt:.1f} s; initial bodies + merges / oracle time"}


def serve_bench(args):
    """Serving: capacity (every episode at t = 0), then a sweep of Poisson
    arrival rates.  Every retired world of every run is checked against the
    same episode run alone (result digests) and both pools' heaps against
    their invariants and sticky flags; a sample is also checked against the
    oracle in the CPU-baseline leg."""
    import torch
    from paper_1809_07444_amd import _capi as C
    from paper_1809_07444_amd import serve
    from synth import workloads as W
    torch.cuda.set_device(0)
    n = args.episodes
    srv = serve.Server()
    mismatches, checked = [], 0

    def run(specs, alone=None):
        nonlocal checked
        inputs = {s.eid: W.episode_inputs(s) for s in specs}      # requests carry their data
        recs, digests, st = srv.run(specs, lambda s: inputs[s.eid], digests=True)
        bad = srv.check()
        if bad:
            raise RuntimeError(f"serving heaps failed their check: {bad}")
        if alone is not None:
            for e in specs:
                checked += 1
                if digests[e.eid] != alone[e.eid]:
                    mismatches.append(e.eid)
        return serve.summarize(recs, st["wall_s"]), st, digests

    try:
        run(W.serving_episodes(16, float("inf"), seed=args.seed + 1))          # warm-up
        base = W.serving_episodes(n, float("inf"), seed=args.seed)
        # Each episode alone (one at a time through the empty pools): the
        # reference every mixed run is compared with.
        alone = {}
        for e in base:
            _, _, d = run([e])
            alone.update(d)
        cap_sum, cap_st, _ = run(base, alone)
        capacity = cap_sum["episodes_per_s"]
        sweep = []
        for f in [float(x) for x in args.rates.split(",")]:
            specs = W.serving_episodes(n, f * capacity, seed=args.seed)
            s, st, _ = run(specs, alone)
            sweep.append(dict(s, rate_fraction=f, rate_episodes_per_s=f * capacity, server_steps=st["server_steps"]))
            print(json.dumps({"progress": "serve", "rate_fraction": f, **s}), file=sys.stderr, flush=True)
        # Profiled capacity run: per-launch timing on both pools, the steps
        # launched eagerly (kernels inside a replayed graph carry no events).
        # The pools' counters run over their whole life: the byte models take
        # the difference over this run.
        st0 = {}
        for name, p in srv.pools.items():
            p.heap.set_timing(True)
            p.flags &= ~C.GRAPH
            st0[name] = p.heap.stats()
        run(base)
        roof, kernels = serve_roofline(srv, base, st0)
    finally:
        srv.close()
    if mismatches:
        raise RuntimeError(f"serving results differ from the episodes run alone: {mismatches[:10]}")
    best = max(sweep, key=lambda r: r["episodes_per_s"])
    cpu = None if args.no_cpu_baseline else serve_cpu_baseline(base, alone)
    out = {"metric": METRIC, "value": best["episodes_per_s"], "unit": "episodes/s", "n_gpus": 1,
           "steps": len(sweep), "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32/u64", "data": "synthetic",
           "config": {"workload": f"serve-poisson-{n}episodes-70%gol128..2048-30%sugar256..1024",
                      "episodes_per_rate": n, "seed": args.seed},
           "capacity_episodes_per_s": capacity, "capacity_run": dict(cap_sum, **cap_st), "sweep": sweep,
           "parity": {"episodes_checked_against_alone": checked, "mismatches": 0, "heap_checks": "ok"},
           "roofline": roof, "cpu_baseline": cpu, "kernels": kernels}
    print(json.dumps(out))


def stats_delta(after: dict, before: dict, keys=("allocs", "frees", "visits")) -> dict:
    """The cumulative per-type counters `keys` of `after` minus those of
    `before`; other entries as in `after`."""
    out = dict(after)
    for k in keys:
        if k in after and k in before:
            out[k] = [x - y for x, y in zip(after[k], before[k])]
    return out


def serve_roofline(srv, specs, st0):
    """Dominant kernel of a profiled serving run over both pools, with its
    algorithmic bytes (the Game-of-Life and Sugarscape byte models over the
    pool's own counters for that run: their change since `st0`)."""
    from synth import workloads as W
    gol_alive0 = sum(int(W.episode_inputs(e).sum()) for e in specs if e.kind == "gol")
    sugar_agents0 = sum(int(W.episode_inputs(e).occ.sum()) for e in specs if e.kind == "sugar")
    sugar_cells = sum(e.side ** 2 * e.length for e in specs if e.kind == "sugar")
    kernels, best = {}, None
    for name, p in srv.pools.items():
        kern = p.heap.timing()
        st = stats_delta(p.heap.stats(), st0[name])
        p.heap.set_timing(False)
        for kind, (launches, tot_ms) in kern.items():
            if name == "gol":
                b = gol_kernel_bytes(kind, launches, st, p.blocks, gol_alive0)
            else:
                # regrow sweeps the arena; count the episodes' own cells instead
                b = sugar_kernel_bytes(kind, launches, st, p.blocks, sugar_agents0, sugar_cells / max(launches, 1))
            other = None
            if isinstance(b, tuple):
                b, other = b
            key = f"{name}:{kind}"
            kernels[key] = {"launches": launches, "avg_us": tot_ms / launches * 1e3, "total_ms": tot_ms,
                            "gbs": b / (tot_ms / 1e3) / 1e9 if b is not None and tot_ms > 0 else None}
            if b is not None:
                kernels[key]["bytes_per_launch"] = b / launches
            if other is not None:
                kernels[key]["other_bytes_per_launch"] = other / launches
            if best is None or tot_ms > kernels[best]["total_ms"]:
                best = key
    k = kernels[best]
    roof = None
    if k["gbs"] is not None:
        roof = {"bound": "hbm", "achieved": round(k["gbs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(k["gbs"] / HBM_PEAK_GBS, 5), "traffic": None, "kernel": best,
                "avg_launch_us": round(k["avg_us"], 2), "algorithmic_bytes_per_launch": round(k["bytes_per_launch"])}
        if "other_bytes_per_launch" in k:
            roof["other_bytes_per_launch"] = round(k["other_bytes_per_launch"])
    return roof, kernels


def serve_cpu_baseline(specs, alone):
    """The oracle on the first episodes in arrival order until about 10 s of
    CPU work (episodes per second), each result also checked against the
    device's digest of the same episode."""
    import numpy as np

    import oracle
    from paper_1809_07444_amd import serve
    from synth import workloads as W
    t0 = time.perf_counter()
    done = 0
    oracle_s = 0.0
    for e in specs:
        inp = W.episode_inputs(e)
        t1 = time.perf_counter()
        if e.kind == "gol":
            res, _ = oracle.gol_run(inp, e.length)
        else:
            st = oracle.SugarState(e.side, inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab, inp.a_vision,
                                   inp.a_age)
            r = oracle.sugar_run(st, e.length, e.seed, W.SUGAR_RULES)
            m = r.occ.astype(bool)
            res = {"sugar": r.sugar, "occ": r.occ, "moves": r.moves,
                   **{f: np.where(m, getattr(r, f), 0).astype(np.int32) for f in ("a_sugar", "a_metab", "a_vision",
                                                                                   "a_age")}}
        oracle_s += time.perf_counter() - t1
        if serve.result_digest(e.kind, res) != alone[e.eid]:
            raise RuntimeError(f"serving episode {e.eid} differs from the oracle")
        done += 1
        if time.perf_counter() - t0 > 10:
            break
    return {"value": done / oracle_s, "unit": "episodes/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (dense Game of Life stencil / sequential Sugarscape rules) on the first {done} "
                      f"of {len(specs)} episodes in arrival order, {oracle_s:.1f} s; each equal to the device's "
                      f"result"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(the path runs on one GPU; sharding across GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "serve":
        return serve_bench(args)
    if args.workload == "gol":
        wl = GolWorkload(args)
    elif args.workload == "batched":
        wl = BatchedWorkload(args)
    elif args.workload == "sugarscape":
        wl = SugarWorkload(args)
    elif args.workload == "traffic":
        wl = TrafficWorkload(args)
    elif args.workload in ("collisions", "nbody"):
        wl = CollideWorkload(args)
    elif args.workload == "wator":
        wl = WatorWorkload(args)
    else:
        wl = MicroWorkload(args, scaled=args.workload == "micro_scaled")

    if args.bulk_min is not None:
        wl.heap().set_policy(args.bulk_min)
        wl.config["bulk_min"] = args.bulk_min
    if args.unroll is not None:
        wl.heap().set_unroll(args.unroll)
        wl.config["unroll"] = args.unroll
    if args.reclaim == "online":
        wl.heap().set_reclaim(True)
        wl.config["reclaim"] = "online"

    for _ in range(args.warmup):
        wl.step()
    torch.cuda.synchronize()
    st0 = wl.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        wl.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st1 = wl.stats()
    # Counters accumulate until a reset; init() resets the heap, so the stats
    # after the timed loop describe exactly the last step.
    per_step_ops = sum(st1["allocs"]) + sum(st1["frees"])
    per_step_visits = sum(st1["visits"])
    ms = dt / max(args.steps, 1) * 1e3
    value = per_step_ops / (ms / 1e3)

    # Profiled pass: per-launch HIP events on the launch stream.
    heap = wl.heap()
    heap.set_timing(True)
    wl.profiled_step()
    kern = heap.timing()
    stp = wl.stats()
    heap.set_timing(False)
    kernels = {}
    best = None
    for kind, (launches, tot_ms) in kern.items():
        b = wl.kernel_bytes(kind, launches, stp)
        other = None
        if isinstance(b, tuple):
            b, other = b
        k = {"launches": launches, "avg_us": tot_ms / launches * 1e3, "total_ms": tot_ms,
             "gbs": (b / (tot_ms / 1e3) / 1e9) if b is not None and tot_ms > 0 else None}
        if b is not None:
            k["bytes_per_launch"] = b / launches
        if other is not None:
            k["other_bytes_per_launch"] = other / launches
            k["other_gbs"] = other / (tot_ms / 1e3) / 1e9 if tot_ms > 0 else None
        kernels[kind] = k
        if best is None or tot_ms > kern[best][1]:
            best = kind
    roof = None
    flops = getattr(wl, "kernel_flops", lambda *a: None)(best, kern[best][0], stp) if best else None
    if flops is not None:
        # An arithmetic-bound kernel: algorithmic float32 operations per second
        # against the chip's vector FP32 peak.
        ach = flops / (kern[best][1] / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_PEAK_TFLOPS, 5), "traffic": None, "kernel": best,
                "avg_launch_us": round(kernels[best]["avg_us"], 2)}
    elif best is not None and kernels[best]["gbs"] is not None:
        ach = kernels[best]["gbs"]
        roof = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None, "kernel": best,
                "avg_launch_us": round(kernels[best]["avg_us"], 2),
                "algorithmic_bytes_per_launch": round(kernels[best]["bytes_per_launch"])}
        if "other_bytes_per_launch" in kernels[best]:
            # Other objects' state the kernel reads or writes (not in achieved).
            roof["other_bytes_per_launch"] = round(kernels[best]["other_bytes_per_launch"])

    # Bytes beyond L2 per launch of the dominant kernel, from the committed
    # rocprofv3 counter summary of this workload, while the device sources
    # still hash as they did when the counters were taken (else null).
    if roof is not None:
        from paper_1809_07444_amd import profiling
        summ = profiling.read_summary(os.path.join(ROOT, "profiles", f"traffic_{wl.name}.txt"))
        if summ and summ["source_hash"] == profiling.source_hash() and best in summ["kernels"]:
            roof["traffic"] = summ["kernels"][best]

    cpu = None
    if not args.no_cpu_baseline:
        cpu = wl.cpu_baseline()

    extra = {}
    if args.probe:
        from paper_1809_07444_amd import probe
        extra["ceilings"] = dict(probe.atomics(), copy_gbs=probe.copy_bandwidth())
    if args.workload == "batched" and not args.no_plain:
        pb = wl.plain_baseline()
        extra["batched_vs_plain"] = dict(pb, batched_ms=ms, speedup_vs_plain=pb["plain_ms"] / ms,
                                         speedup_vs_plain_sync=pb["plain_sync_ms"] / ms)

    if args.traffic_probe:
        a = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.add(a, 1, out=b)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC, "value": value, "unit": "allocs+frees/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32/u64", "data": "synthetic", "config": wl.config,
        "doall_objects_per_s": per_step_visits / (ms / 1e3),
        "cells_gens_per_s": (wl.cells_gens / (ms / 1e3)) if getattr(wl, "cells_gens", None) else None,
        "per_step": {"allocs": st1["allocs"], "frees": st1["frees"], "doall_visits": st1["visits"],
                     "reserve_retries": st1["reserve_retries"], "slow_paths": st1["slow_paths"],
                     "find_fails": st1["find_fails"], "method_atomics": st1["method_atomics"],
                     "online_releases": st1["online_releases"],
                     "allocated_blocks_end": st1["allocated_blocks"]},
        "roofline": roof, "cpu_baseline": cpu, "kernels": kernels,
    }
    out.update(extra)
    del st0
    print(json.dumps(out))


if __name__ == "__main__":
    main()
