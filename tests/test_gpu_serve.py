"""Serving with continuous batching: episodes admitted by free-block budget
into resident world pools and stepped together.  Every result must equal the
oracle's and the same episode run alone (tolerance 0: the work is integer)."""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import serve  # noqa: E402
from synth import workloads as W  # noqa: E402

RULES = W.SUGAR_RULES


def small_specs(n=24, rate=float("inf"), seed=11):
    return W.serving_episodes(n, rate, seed=seed, gol_sides=(12, 64), gol_lengths=(3, 40), sugar_sides=(10, 40),
                              sugar_agents=(20, 400), sugar_steps=12)


def small_server(**kw):
    # Small pools so that episodes must wait for each other's blocks.
    args = dict(gol_blocks=1024, gol_slots=8, gol_arena=1 << 15, sugar_blocks=256, sugar_slots=4,
                sugar_arena=1 << 13)
    args.update(kw)
    return serve.Server(**args)


def check_against_oracle(spec, res):
    inp = W.episode_inputs(spec)
    if spec.kind == "gol":
        exp, _ = oracle.gol_run(inp, spec.length)
        assert np.array_equal(res, exp)
    else:
        st = oracle.SugarState(spec.side, inp.sugar, inp.cap, inp.occ, inp.a_sugar, inp.a_metab, inp.a_vision,
                               inp.a_age)
        ref = oracle.sugar_run(st, spec.length, spec.seed, RULES)
        assert np.array_equal(res["sugar"], ref.sugar) and np.array_equal(res["occ"], ref.occ)
        m = ref.occ.astype(bool)
        for f in ("a_sugar", "a_metab", "a_vision", "a_age"):
            assert np.array_equal(res[f][m], getattr(ref, f)[m])
        assert res["moves"] == ref.moves


def same(a, b):
    if isinstance(a, dict):
        return all(np.array_equal(a[k], b[k]) if isinstance(a[k], np.ndarray) else a[k] == b[k] for k in a)
    return np.array_equal(a, b)


def test_mix_equals_alone_and_oracle():
    specs = small_specs()
    srv = small_server()
    records, results, stats = srv.run(specs, W.episode_inputs)
    assert len(records) == len(specs)
    # Continuous batching: some episode was admitted while another was resident,
    # and some had to wait for blocks (admitted after arrival at t=0).
    by = {r.eid: r for r in records}
    overlap = any(a.admitted < b.done and b.admitted < a.done for a in records for b in records if a.eid < b.eid)
    assert overlap
    assert any(r.admitted > 0 for r in records)
    for spec in specs:
        check_against_oracle(spec, results[spec.eid])
    for p in srv.pools.values():
        assert p.budget == p.blocks and not p.resident
        assert p.heap.check() == {}
    srv.close()
    # Each episode alone, in a fresh server, gives the identical result.
    for spec in specs[:8]:
        alone = small_server()
        _, res_alone, _ = alone.run([spec], W.episode_inputs)
        assert same(results[spec.eid], res_alone[spec.eid])
        alone.close()
    assert by


def test_poisson_arrivals_complete():
    specs = small_specs(n=16, rate=200.0, seed=5)
    srv = small_server(graph=False)
    records, results, stats = srv.run(specs, W.episode_inputs)
    assert sorted(r.eid for r in records) == [s.eid for s in specs]
    for r in records:
        assert r.admitted >= r.arrival - 1e-9 and r.done >= r.admitted
    s = serve.summarize(records, stats["wall_s"])
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
    for spec in specs[:6]:
        check_against_oracle(spec, results[spec.eid])
    srv.close()


def test_serving_config_sizes_against_oracle_digests():
    # The serving configuration at its own sizes, on the server's default
    # pools (2^21 Game-of-Life blocks, 256 slots, a 2^25-cell arena; 2^19
    # Sugarscape blocks, 64 slots, a 2^23-cell arena): ten episodes of the
    # Poisson stream plus a 2048^2 Game of Life of 240 generations and a
    # 1024^2 Sugarscape world of 150,000 agents, arriving while others run.
    # Every retired world equals the oracle's (stored digests written from
    # oracle/ by tests/golden/make_golden.py) and the same episode run alone.
    import json
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import episode_digest
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "serving_10plus2_seed24301.json")))
    specs = [W.EpisodeSpec(e["eid"], e["kind"], e["side"], e["length"], int(e["seed"]), e["agents"], e["arrival"])
             for e in gold["episodes"]]
    assert max(s.side for s in specs if s.kind == "gol") == 2048
    assert max(s.agents for s in specs if s.kind == "sugar") >= 100_000
    want = {e["eid"]: {k: v for k, v in e.items() if k not in ("eid", "kind", "side", "length", "seed", "agents",
                                                               "arrival")} for e in gold["episodes"]}
    srv = serve.Server()
    records, results, _ = srv.run(specs, W.episode_inputs)
    assert sorted(r.eid for r in records) == sorted(s.eid for s in specs)
    overlap = any(a.admitted < b.done and b.admitted < a.done for a in records for b in records if a.eid < b.eid)
    assert overlap
    for spec in specs:
        assert episode_digest(spec.kind, results[spec.eid]) == want[spec.eid], spec
    assert srv.check() == {}
    for p in srv.pools.values():
        assert p.budget == p.blocks and not p.resident
    # Alone: one episode at a time through the same (now empty) pools.
    for spec in specs:
        _, alone, _ = srv.run([dataclasses.replace(spec, arrival=0.0)], W.episode_inputs, digests=True)
        assert alone[spec.eid] == serve.result_digest(spec.kind, results[spec.eid]), spec
    assert srv.check() == {}
    srv.close()
