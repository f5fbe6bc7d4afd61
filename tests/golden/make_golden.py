"""Writes the stored expected values of the large parity cases.

Every value here comes from the oracle (oracle/) run on the seeded inputs of
synth/; nothing is taken from the device path.  Usage:
    python tests/golden/make_golden.py [batched|sugarscape|serving|wator|collisions|nbody|all]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from synth import workloads as W  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def batched(n_worlds=256, generations=100, seed=24301):
    inp = W.batch_inputs(n_worlds, generations, seed=seed)
    worlds = []
    t0 = time.time()
    for i, (side, g0) in enumerate(zip(inp.sides.tolist(), inp.grids)):
        final, c = oracle.gol_run(g0, generations)
        worlds.append({"side": side, "sha256": digest(final.astype(np.uint8)), "population": int(final.sum()),
                       "initial_population": int(g0.sum()), "candidates": int(c[:, 0].sum()),
                       "births": int(c[:, 1].sum()), "deaths": int(c[:, 2].sum())})
    out = {"case": f"gol batched: {n_worlds} worlds, sides log-uniform 64..1024, Bernoulli(0.1), "
                   f"{generations} generations, seed {seed}",
           "source": "oracle.gol_run (dense B3/S23 torus) on synth.workloads.batch_inputs",
           "n_worlds": n_worlds, "generations": generations, "seed": seed,
           "total_cells": int(sum(w["side"] ** 2 for w in worlds)), "worlds": worlds,
           "oracle_seconds": round(time.time() - t0, 1)}
    path = os.path.join(HERE, f"gol_batched_{n_worlds}w_{generations}g_seed{seed}.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path, out["oracle_seconds"], "s")


def sugarscape(side=2048, n_agents=1 << 20, steps=500, seed=24301, every=100):
    inp = W.sugar_inputs(side, n_agents, seed=seed)
    rules = W.SUGAR_RULES
    s = oracle.SugarState(side, inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab, inp.a_vision, inp.a_age)
    checkpoints = []
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        s = oracle.sugar_run(s, k, seed, rules, step0=done)
        done += k
        m = s.occ.astype(bool)
        checkpoints.append({
            "step": done, "agents": int(m.sum()), "births": s.births, "deaths": s.deaths, "moves": s.moves,
            "sugar_grid_sha256": digest(s.sugar), "occ_sha256": digest(s.occ),
            "agents_sha256": digest(np.stack([np.where(m, s.a_sugar, 0), np.where(m, s.a_metab, 0),
                                              np.where(m, s.a_vision, 0), np.where(m, s.a_age, 0)]).astype(np.int32)),
            "total_agent_sugar": int(s.a_sugar[m].sum()), "total_cell_sugar": int(s.sugar.sum())})
        print(checkpoints[-1]["step"], checkpoints[-1]["agents"], round(time.time() - t0, 1), flush=True)
    out = {"case": f"sugarscape: {side}x{side} torus, {n_agents} agents, {steps} steps, seed {seed}",
           "source": "oracle.sugar_run on synth.workloads.sugar_inputs", "rules": rules, "side": side,
           "n_agents": n_agents, "steps": steps, "seed": seed, "checkpoints": checkpoints,
           "oracle_seconds": round(time.time() - t0, 1)}
    path = os.path.join(HERE, f"sugarscape_{side}_{n_agents}a_{steps}s_seed{seed}.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path, out["oracle_seconds"], "s")


def episode_digest(kind: str, res) -> dict:
    """Canonical digest of an episode's final state: for the Game of Life the
    grid (uint8, row-major); for Sugarscape the sugar grid (int32), the
    occupancy (uint8), the agents' sugar, metabolism, vision and age per cell
    (int32, 0 where no agent stands) and the number of moves."""
    if kind == "gol":
        g = np.ascontiguousarray(res, dtype=np.uint8)
        return {"grid_sha256": digest(g), "population": int(g.sum())}
    m = np.asarray(res["occ"]).astype(bool).ravel()
    agents = np.stack([np.where(m, np.asarray(res[f]).ravel(), 0) for f in ("a_sugar", "a_metab", "a_vision", "a_age")])
    return {"sugar_sha256": digest(np.asarray(res["sugar"], dtype=np.int32).ravel()),
            "occ_sha256": digest(np.asarray(res["occ"], dtype=np.uint8).ravel()),
            "agents_sha256": digest(agents.astype(np.int32)), "final_agents": int(m.sum()), "moves": int(res["moves"])}


def serving_case(seed=24301, rate=40.0, n=10):
    """The serving parity case at the sizes of the serving configuration:
    the first n episodes of the Poisson stream (70 % Game of Life, side
    128..2048, 50..300 generations; 30 % Sugarscape, side 256..1024, 10k..200k
    agents, 100 steps) plus the two largest shapes the configuration allows,
    a 2048^2 Game of Life of 240 generations and a 1024^2 Sugarscape world of
    150,000 agents."""
    from synth import rng
    specs = W.serving_episodes(n, rate, seed=seed)
    big_seeds = rng.hash4(seed, rng.S_EPISODE, 99, np.arange(2, dtype=np.uint64))
    specs.append(W.EpisodeSpec(100, "gol", 2048, 240, int(big_seeds[0]), 0, 0.02))
    specs.append(W.EpisodeSpec(101, "sugar", 1024, 100, int(big_seeds[1]), 150_000, 0.05))
    eps = []
    t0 = time.time()
    for e in specs:
        inp = W.episode_inputs(e)
        if e.kind == "gol":
            final, _ = oracle.gol_run(inp, e.length)
            d = episode_digest("gol", final)
        else:
            st = oracle.SugarState(e.side, inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab, inp.a_vision,
                                   inp.a_age)
            ref = oracle.sugar_run(st, e.length, e.seed, W.SUGAR_RULES)
            d = episode_digest("sugar", {"sugar": ref.sugar, "occ": ref.occ, "a_sugar": ref.a_sugar,
                                         "a_metab": ref.a_metab, "a_vision": ref.a_vision, "a_age": ref.a_age,
                                         "moves": ref.moves})
        eps.append({"eid": e.eid, "kind": e.kind, "side": e.side, "length": e.length, "seed": str(e.seed),
                    "agents": e.agents, "arrival": float(e.arrival), **d})
        print(e.eid, e.kind, e.side, e.length, e.agents, round(time.time() - t0, 1), flush=True)
    out = {"case": f"serving: first {n} episodes of the Poisson stream at {rate}/s (seed {seed}) plus a 2048^2 "
                   f"Game of Life x 240 generations and a 1024^2 Sugarscape world with 150,000 agents x 100 steps",
           "source": "oracle.gol_run / oracle.sugar_run on synth.workloads.episode_inputs", "rules": W.SUGAR_RULES,
           "seed": seed, "rate": rate, "episodes": eps, "oracle_seconds": round(time.time() - t0, 1)}
    path = os.path.join(HERE, f"serving_{n}plus2_seed{seed}.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path, out["oracle_seconds"], "s")


def wator(side=2048, steps=200, seed=24301, every=50):
    inp = W.wator_inputs(side, seed=seed)
    rules = W.WATOR_RULES
    s = oracle.WatorState(inp.kind, inp.age, inp.energy)
    checkpoints = []
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        s = oracle.wator_run(s, k, seed, rules, step0=done)
        done += k
        checkpoints.append({
            "step": done, "fish": int((s.kind == 1).sum()), "sharks": int((s.kind == 2).sum()),
            "fish_born": s.fish_born, "sharks_born": s.sharks_born, "fish_eaten": s.fish_eaten,
            "sharks_starved": s.sharks_starved, "kind_sha256": digest(s.kind), "age_sha256": digest(s.age),
            "energy_sha256": digest(s.energy)})
        print(checkpoints[-1]["step"], checkpoints[-1]["fish"], checkpoints[-1]["sharks"],
              round(time.time() - t0, 1), flush=True)
    out = {"case": f"wa-tor: {side}x{side} sea, fish 0.30, sharks 0.05, {steps} steps, seed {seed}",
           "source": "oracle.wator_run on synth.workloads.wator_inputs", "rules": rules, "side": side,
           "steps": steps, "seed": seed,
           "initial": {"fish": int((inp.kind == 1).sum()), "sharks": int((inp.kind == 2).sum())},
           "checkpoints": checkpoints, "oracle_seconds": round(time.time() - t0, 1)}
    path = os.path.join(HERE, f"wator_{side}_{steps}s_seed{seed}.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path, out["oracle_seconds"], "s")


def collisions(n=65536, steps=20, seed=24301, every=5, merge=True):
    inp = W.collide_inputs(n, seed=seed, box=32.0)
    params = W.COLLIDE_PARAMS if merge else dict(W.COLLIDE_PARAMS, r2_merge=0.0)
    s = oracle.CollideState(inp.x, inp.y, inp.vx, inp.vy, inp.m)
    checkpoints = []
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        s = oracle.collide_run(s, k, params)
        done += k
        cp = {"step": done, "merges": int(s.merges), "live": int((s.m > 0).sum())}
        for f in ("x", "y", "vx", "vy", "m"):
            cp[f + "_sha256"] = digest(getattr(s, f).view(np.uint32))
        checkpoints.append(cp)
        print(done, cp["live"], round(time.time() - t0, 1), flush=True)
    name = "collisions" if merge else "nbody"
    out = {"case": f"{name}: {n} bodies in a 32 x 32 box, {steps} steps, seed {seed}",
           "source": "oracle.collide_run on synth.workloads.collide_inputs", "params": params, "bodies": n,
           "steps": steps, "seed": seed, "checkpoints": checkpoints, "oracle_seconds": round(time.time() - t0, 1)}
    path = os.path.join(HERE, f"{name}_{n}_{steps}s_seed{seed}.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path, out["oracle_seconds"], "s")


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("batched", "all"):
        batched()
    if what in ("sugarscape", "all"):
        sugarscape()
    if what in ("serving", "all"):
        serving_case()
    if what in ("wator", "all"):
        wator()
    if what in ("collisions", "all"):
        collisions()
    if what in ("nbody", "all"):
        collisions(merge=False)
