"""The largest heap the handle format allows, filled to capacity and drained.

A handle is block << 6 | slot in 32 bits and DSOAR_NULL is all ones (slot 63
of block 2^26 - 1), so a heap holds at most 2^26 - 1 blocks of 64 slots:
handles then reach 2^32 - 65, the field data spans 16 GiB and the bitmaps
have 5 levels at width 64 (6 at width 32); blocks of 32 slots too.  Device new fills the heap to
exactly its capacity (Sec. 2.2: a request fails only when no block has room),
the do-all visits every object once, the enumeration and its allocation-free
variant list every block, one more request fails as out of memory, and device
delete plus quiescent reclamation return every block.  About 40 GiB of device
memory per case.
"""
import pytest
import torch

from paper_1809_07444_amd import _capi as C
from paper_1809_07444_amd.heap import Heap

M = (1 << 26) - 1
CHUNK = 1 << 28


def _step(msg):
    print(f"[max heap] {msg}", flush=True)


def _covers_every_slot(h: torch.Tensor, cap: int) -> bool:
    """True when the M * cap handles (block << 6 | slot) are M * cap distinct
    slots: blocks below M, slots below cap, no NULL."""
    n = M * cap
    seen = torch.zeros(n, dtype=torch.bool, device=h.device)
    for i in range(0, n, CHUNK):
        part = h[i:i + CHUNK].to(torch.int64) & 0xFFFFFFFF
        blk, slot = part >> 6, part & 63
        if not bool(((blk < M) & (slot < cap)).all()):  # checked before the values index anything
            return False
        seen[blk * cap + slot] = True
        del part, blk, slot
    ok = bool(seen.all())
    del seen
    return ok


@pytest.mark.gpu
@pytest.mark.parametrize("width,cap", [(64, 64), (32, 64), (64, 32)])
def test_largest_heap_fills_to_capacity_and_drains(width, cap):
    N = M * cap  # 2^32 - 64 objects at 64 slots per block
    full = (1 << cap) - 1 if cap < 64 else -1  # a full block's snapshot, as int64
    _step(f"width {width}, {cap} slots: create {M} blocks")
    heap = Heap(M, cap, [(4,)], bitmap_width=width)
    assert heap.layout().num_levels == (5 if width == 64 else 6)
    try:
        _step(f"width {width}, {cap} slots: {N} device new")
        h = heap.alloc_n(0, N)
        torch.cuda.synchronize()
        st = heap.stats()
        assert st["live"] == [N] and st["allocs"] == [N]
        assert st["allocated_blocks"] == [M] and st["active_blocks"] == [0] and st["free_blocks"] == 0
        _step(f"width {width}, {cap} slots: handle coverage")
        assert _covers_every_slot(h, cap)
        _step(f"width {width}, {cap} slots: do-all visit counts")
        counts = heap.visit_counts(0).view(M, 64)
        visited_once = bool((counts[:, :cap] == 1).all()) and bool((counts[:, cap:] == 0).all())
        del counts
        assert visited_once
        assert heap.enum_count(0) == M
        R, S = heap.enum_arrays(0, M)
        assert torch.equal(R, torch.arange(M, dtype=torch.int32, device=R.device))
        assert bool((S == full).all())
        _step(f"width {width}, {cap} slots: allocation-free enumeration")
        R2 = torch.full((M,), -1, dtype=torch.int32, device=R.device)
        S2 = torch.zeros(M, dtype=torch.int64, device=R.device)
        cnt = torch.full((1,), -1, dtype=torch.int32, device=R.device)
        assert heap.lib.dsoar_enumerate_noalloc(heap.h, 0, R2.data_ptr(), S2.data_ptr(), cnt.data_ptr(),
                                                heap._s()) == C.OK
        torch.cuda.synchronize()
        assert int(cnt.item()) == M and torch.equal(R2, R) and torch.equal(S2, S)
        del R2, S2
        assert heap.check() == {}
        _step(f"width {width}, {cap} slots: one request more")
        extra = heap.alloc_n(0, 64)
        assert bool((extra == -1).all())  # DSOAR_NULL read as int32
        st = heap.stats(raise_sticky=False)
        assert st["oom"] == 1 and st["status"] == C.ERR_OOM and st["live"] == [N]
        _step(f"width {width}, {cap} slots: {N} device delete")
        heap.free_n(h)
        del h
        heap.enumerate(0)  # quiescent reclamation of every emptied block
        st = heap.stats(raise_sticky=False)
        assert st["live"] == [0] and st["frees"] == [N]
        assert st["allocated_blocks"] == [0] and st["active_blocks"] == [0] and st["free_blocks"] == M
        assert st["blocks_returned"] == M and st["double_free"] == 0
        assert heap.check() == {"sticky": "DSOAR_ERR_OOM"}
    finally:
        heap.close()
        del heap
        torch.cuda.empty_cache()
