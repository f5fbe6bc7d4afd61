"""Measured ceilings: agent-scope atomic throughput/latency and streaming copy
bandwidth on the current GPU (the library's probe kernels, timed with events)."""
from __future__ import annotations

import torch

from . import _capi as C


def _time(fn, reps=3):
    s = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    return best


def atomics(waves: int = 65536, iters: int = 64) -> dict:
    lib = C.load()
    words = 8 * waves + 64
    buf = torch.zeros(words, dtype=torch.int64, device="cuda")
    s = int(torch.cuda.current_stream().cuda_stream)
    out = {}
    for mode, name, w in ((0, "distinct_atomics_per_s", waves), (2, "same_address_atomics_per_s", 4096)):
        run = lambda: C.check(lib.dsoar_probe_atomics(buf.data_ptr(), words, mode, iters, w, s), "probe")
        run()
        out[name] = w * iters / _time(run)
    for mode, name in ((1, "dependent_atomic_latency_us"), (3, "dependent_load_latency_us")):
        run = lambda: C.check(lib.dsoar_probe_atomics(buf.data_ptr(), words, mode, 256, 1, s), "probe")
        run()
        out[name] = _time(run) / 256 * 1e6
    return out


def copy_bandwidth(mib: int = 1024) -> float:
    lib = C.load()
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    s = int(torch.cuda.current_stream().cuda_stream)
    run = lambda: C.check(lib.dsoar_probe_copy(a.data_ptr(), b.data_ptr(), n, s), "probe")
    run()
    return 2 * n / _time(run) / 1e9
