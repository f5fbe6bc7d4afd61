"""Alloc/do-all microbenchmark on the device against the oracle: bit-exact
final objects (compared by id, since slot placement may differ) and exact
churn counts."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd import apps  # noqa: E402
from synth import workloads as W  # noqa: E402


def compare(inp, res):
    ref = oracle.micro_run(inp)
    assert np.array_equal(res.present.astype(bool), ref.present.astype(bool))
    p = ref.present.astype(bool)
    assert np.array_equal(res.x[p].view(np.uint32), ref.x[p].view(np.uint32))
    assert np.array_equal(res.v[p].view(np.uint32), ref.v[p].view(np.uint32))
    st = res.stats
    assert st["status"] == C.OK
    assert st["allocs"] == [ref.allocs] and st["frees"] == [ref.frees]
    assert st["live"] == [int(p.sum())]


def test_micro_full_config():
    # Heap of 4096 blocks x 64 slots, 65,536 objects, 10 steps.
    inp = W.micro_inputs(65536, 10)
    res = apps.micro_run(inp, 4096, 64)
    compare(inp, res)
    assert res.stats["allocs"] == [283996] and res.stats["frees"] == [218460]


@pytest.mark.parametrize("n,steps,seed,cap,flags", [
    (1000, 3, 1, 64, C.DO_PERSISTENT), (4099, 4, 2, 64, C.DO_PLAIN), (4099, 4, 3, 32, C.DO_PERSISTENT),
    (1, 2, 4, 64, C.DO_PERSISTENT), (0, 2, 5, 64, C.DO_PERSISTENT), (20000, 5, 24301, 32, C.DO_PLAIN),
])
def test_micro_ragged(n, steps, seed, cap, flags):
    inp = W.micro_inputs(n, steps, seed=seed)
    blocks = max(4, 4 * (-(-max(n, 1) // cap)))
    res = apps.micro_run(inp, blocks, cap, flags)
    compare(inp, res)


def test_micro_scaled_full_config():
    # The HBM-bound configuration the benchmark times: 2^22 blocks of 64 slots,
    # 2^26 objects (16 per block on average), 2 steps, persistent do-alls.
    inp = W.micro_inputs(16 << 22, 2)
    res = apps.micro_run(inp, 1 << 22, 64)
    compare(inp, res)
