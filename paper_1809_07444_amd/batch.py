"""Batched worlds: many independent Game-of-Life worlds of uneven size in one
heap, one persistent do-all per phase covering all of them, each generation
replayed from a HIP graph; the per-world "plain" baseline; and the autotuner
that picks block capacity, bitmap fan-out (container width), do-all launch
shape, allocation policy and where bitmap searches start.

Every configuration computes the same result (the worlds are independent and
the update is synchronous); the tuner only measures time."""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time
from dataclasses import asdict, dataclass

import torch

from . import _capi as C
from .apps import GameOfLife

NEVER = 0xFFFFFFFF


@dataclass(frozen=True)
class TuneConfig:
    capacity: int = 64         # slots per block; 0 = per type by object size
    wg_threads: int = 256
    wgs_per_cu: int = 8
    bulk_min: int = 0          # 0 = whole free blocks first; NEVER = active blocks first (dense)
    bitmap_width: int = 64     # container width of the block-state bitmaps (fan-out 64 or 32)
    search: int = C.SEARCH_HASHED  # where bitmap searches start (hashed, lowest, per XCD)

    def apply(self, heap):
        heap.set_launch(self.wg_threads, self.wgs_per_cu)
        heap.set_policy(self.bulk_min)
        heap.set_search(self.search)


# Capacity and bitmap width shape the heap itself (a new heap per pair); the
# other dimensions are settings of one heap.
DEFAULT_SPACE = {
    "capacity": [64, 32, 0],
    "bitmap_width": [64, 32],
    "wg_threads": [256, 1024],
    "wgs_per_cu": [2, 4, 8, 16],
    "bulk_min": [0, NEVER],
    "search": [C.SEARCH_HASHED, C.SEARCH_XCD],
}


def workload_key(grids, generations: int, space: dict | None = None) -> str:
    """Cache key: the worlds, the generations timed and the search space."""
    h = hashlib.sha256()
    for g in grids:
        h.update(str(g.shape).encode())
        h.update(hashlib.sha256(g.tobytes()).digest())
    h.update(str(generations).encode())
    h.update(json.dumps(space or DEFAULT_SPACE, sort_keys=True).encode())
    return h.hexdigest()[:16]


class BatchedGol:
    """All worlds in one heap; generations replayed from a captured graph."""

    def __init__(self, grids, cfg: TuneConfig = TuneConfig(), graph: bool = True, device="cuda"):
        self.cfg = cfg
        self.gol = GameOfLife(grids, capacity=cfg.capacity, device=device, bitmap_width=cfg.bitmap_width)
        cfg.apply(self.gol.heap)
        self.flags = C.DO_PERSISTENT | (C.GOL_GRAPH if graph else 0)

    def run(self, generations: int):
        self.gol.init()
        self.gol.step(generations, self.flags)

    def read(self):
        return self.gol.read()

    def stats(self):
        return self.gol.heap.stats()

    def synchronize(self):
        self.gol.synchronize()


class PlainGol:
    """Baseline: every world has its own heap and its own launches, run one
    world after the other on one stream.  sync=True reads each enumeration
    count back to size the do-all grid (a host round trip per do-all)."""

    def __init__(self, grids, capacity: int = 64, sync: bool = False, device="cuda"):
        self.stream = torch.cuda.Stream(device=device)
        self.worlds = [GameOfLife([g], capacity=capacity, stream=self.stream, device=device) for g in grids]
        self.flags = C.DO_PLAIN if sync else C.DO_PERSISTENT

    def run(self, generations: int):
        for w in self.worlds:
            w.init()
            w.step(generations, self.flags)

    def read(self):
        return [w.read()[0] for w in self.worlds]

    def stats(self):
        tot = None
        for w in self.worlds:
            st = w.heap.stats()
            if tot is None:
                tot = {k: (list(v) if isinstance(v, list) else v) for k, v in st.items()}
            else:
                for k, v in st.items():
                    if isinstance(v, list):
                        tot[k] = [a + b for a, b in zip(tot[k], v)]
        return tot

    def synchronize(self):
        self.stream.synchronize()


def _time_run(runner, generations: int, reps: int = 1) -> float:
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runner.run(generations)
        runner.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def autotune(grids, generations: int = 10, space: dict | None = None, cache_path: str | None = None,
             device="cuda", log=None) -> tuple[TuneConfig, list]:
    """Measures every configuration of `space` on `generations` generations of
    the batch (after a warm-up run that also captures the graph) and returns
    the fastest, with the table of all.  Results are cached by workload."""
    space = space or DEFAULT_SPACE
    key = workload_key(grids, generations, space)
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
        if key in cache:
            ent = cache[key]
            return TuneConfig(**ent["best"]), ent["table"]
    table = []
    for cap, width in itertools.product(space["capacity"], space.get("bitmap_width", [64])):
        b = BatchedGol(grids, TuneConfig(capacity=cap, bitmap_width=width), device=device)
        for wg, per_cu, bulk, search in itertools.product(space["wg_threads"], space["wgs_per_cu"],
                                                          space["bulk_min"], space.get("search", [C.SEARCH_HASHED])):
            cfg = TuneConfig(cap, wg, per_cu, bulk, width, search)
            cfg.apply(b.gol.heap)
            b.cfg = cfg
            _time_run(b, 1)  # captures the graph for this configuration
            t = _time_run(b, generations, reps=2)
            st = b.stats()
            table.append({"config": asdict(cfg), "seconds": t, "oom": st["oom"]})
            if log:
                log(f"autotune {asdict(cfg)} {t * 1e3:.2f} ms")
        del b
        torch.cuda.empty_cache()
    ok = [r for r in table if not r["oom"]]
    best = TuneConfig(**min(ok, key=lambda r: r["seconds"])["config"])
    if cache_path:
        cache = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        cache[key] = {"best": asdict(best), "table": table, "generations": generations}
        json.dump(cache, open(cache_path, "w"), indent=1)
    return best, table
