"""Do-all with several blocks per wavefront pass (the load phase of every block
of a pass runs before any apply): each live object is visited exactly once
(I8), delete-if leaves exactly the expected objects, and the microbenchmark
equals the oracle, for every pass width and launch shape."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd import apps  # noqa: E402
from paper_1809_07444_amd.heap import Heap  # noqa: E402
from synth import workloads as W  # noqa: E402


def populated_heap(unroll, wg, per_cu, seed=7):
    # 4096 blocks; about 3,100 allocated after the deletes, so that with one
    # 64-lane workgroup per CU every wavefront gets 8 or more blocks.
    M = 4096
    heap = Heap(M, 64, [(4, 8)])
    heap.set_launch(wg, per_cu)
    heap.set_unroll(unroll)
    rng = np.random.default_rng(seed)
    h = heap.alloc_n(0, 200000)
    hn = h.cpu().numpy().view(np.uint32)
    assert (hn != C.NULL).all()
    # field 0 = a key per object: its position in allocation order
    keys = np.arange(len(hn), dtype=np.int32)
    heap.field_write(0, 0, h, torch.tensor(keys, device="cuda"))
    kill = hn[rng.random(len(hn)) < 0.4]
    heap.free_n(torch.tensor(kill.view(np.int32), device="cuda"))
    live = np.setdiff1d(hn, kill)
    return heap, hn, live


@pytest.mark.parametrize("unroll,wg,per_cu", [(1, 64, 1), (2, 64, 1), (4, 64, 1), (8, 64, 1), (8, 256, 8),
                                              (4, 1024, 2)])
def test_visits_exactly_once(unroll, wg, per_cu):
    heap, _, live = populated_heap(unroll, wg, per_cu)
    counts = heap.visit_counts(0).cpu().numpy()
    exp = np.zeros(4096 * 64, dtype=np.int32)
    exp[live] = 1
    assert np.array_equal(counts, exp)
    assert heap.check() == {}


@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
def test_delete_if_mod_same_for_every_width(unroll):
    heap, hn, live = populated_heap(unroll, 64, 1)
    heap.delete_if_mod(0, 0, 3, 1)
    torch.cuda.synchronize()
    pos = {int(o): i for i, o in enumerate(hn)}
    keep = {int(o) for o in live if pos[int(o)] % 3 != 1}
    st = heap.stats()
    assert st["live"] == [len(keep)]
    assert st["frees"] == [len(hn) - len(live) + (len(live) - len(keep))]
    counts = heap.visit_counts(0).cpu().numpy()
    assert set(np.nonzero(counts)[0].tolist()) == keep and counts.max() == 1
    assert heap.check() == {}


@pytest.mark.parametrize("unroll,wg,per_cu", [(2, 64, 1), (4, 64, 1), (8, 64, 1), (4, 256, 8)])
def test_micro_every_width_equals_oracle(unroll, wg, per_cu):
    inp = W.micro_inputs(65536, 10)
    mb = apps.MicroBench(inp, 4096, 64)
    mb.heap.set_launch(wg, per_cu)
    mb.heap.set_unroll(unroll)
    mb.run()
    res = mb.result()
    ref = oracle.micro_run(inp)
    p = ref.present.astype(bool)
    assert np.array_equal(res.present.astype(bool), p)
    assert np.array_equal(res.x[p].view(np.uint32), ref.x[p].view(np.uint32))
    assert np.array_equal(res.v[p].view(np.uint32), ref.v[p].view(np.uint32))
    assert res.stats["allocs"] == [ref.allocs] and res.stats["frees"] == [ref.frees]


def test_unroll_rejects_other_widths():
    heap = Heap(64, 64, [(4,)])
    for bad in (0, 3, 5, 16):
        with pytest.raises(RuntimeError):
            heap.set_unroll(bad)
