"""The allocation-free enumeration (dsoar_enumerate_noalloc), called through
the C ABI, against the heap's own enumeration (dsoar_enumerate): the same
count, block list and object-bitmap snapshots, bit for bit, on two calls in
a row, the second on a smaller heap than the first."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd.heap import Heap  # noqa: E402


def churned_heap(num_blocks, n, seed):
    heap = Heap(num_blocks, 64, [(4, 4)])
    rng = np.random.default_rng(seed)
    h = heap.alloc_n(0, n)
    kill = h[torch.from_numpy(rng.random(n) < 0.6).cuda()]
    heap.free_n(kill)
    return heap


def noalloc(heap, t=0):
    M = heap.num_blocks
    R = torch.full((M,), -1, dtype=torch.int32, device="cuda")
    S = torch.zeros(M, dtype=torch.int64, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    rc = heap.lib.dsoar_enumerate_noalloc(heap.h, t, R.data_ptr(), S.data_ptr(), cnt.data_ptr(), heap._s())
    assert rc == C.OK
    torch.cuda.synchronize()
    c = int(cnt.item())
    return c, R[:c].cpu().numpy(), S[:c].cpu().numpy()


def reference(heap, t=0):
    heap.enumerate(t)
    c = heap.enum_count(t)
    R, S = heap.enum_arrays(t, c)
    return c, R[:c].cpu().numpy().copy(), S[:c].cpu().numpy().copy()


@pytest.mark.parametrize("sizes", [((1 << 16, 1 << 21), (4096, 150_000)), ((1 << 20, 1 << 22), (64, 1500))])
def test_noalloc_enumeration_equals_the_heaps_own(sizes):
    for k, (M, n) in enumerate(sizes):
        heap = churned_heap(M, n, seed=k + 1)
        c0, R0, S0 = reference(heap)
        c1, R1, S1 = noalloc(heap)
        assert c0 > 0 and c1 == c0
        assert np.array_equal(R1, R0) and np.array_equal(S1, S0)
        # An allocated block appears once, ascending, with a non-empty snapshot.
        assert (np.diff(R1.astype(np.int64)) > 0).all() and (S1 != 0).all()
        assert heap.check() == {}


def test_noalloc_rejects_bad_arguments():
    heap = churned_heap(256, 3000, seed=9)
    buf = torch.zeros(256 * 3, dtype=torch.int64, device="cuda")
    p = buf.data_ptr()
    assert heap.lib.dsoar_enumerate_noalloc(heap.h, 1, p, p + 2048, p + 4096, heap._s()) == C.ERR_INVALID_ARG
    assert heap.lib.dsoar_enumerate_noalloc(heap.h, 0, None, p, p, heap._s()) == C.ERR_INVALID_ARG
    assert heap.lib.dsoar_enumerate_noalloc(None, 0, p, p, p, None) == C.ERR_INVALID_ARG
