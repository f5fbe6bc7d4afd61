"""Host drivers of the workloads over the C ABI (argument marshalling only)."""
from __future__ import annotations

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
