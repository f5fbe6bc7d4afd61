"""The C-ABI library loads without a GPU and exports every function that
include/dsoar.h declares; host-only entry points validate their arguments."""
import ctypes
import dataclasses
import os
import re

import numpy as np
import pytest

from paper_1809_07444_amd import _capi as C
from paper_1809_07444_amd.heap import make_desc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**(dsoar_[a-z0-9_]+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ["dsoar_heap_create", "dsoar_heap_destroy", "dsoar_parallel_do", "dsoar_heap_stats",
              "dsoar_heap_check", "dsoar_enumerate", "dsoar_alloc_n", "dsoar_free_n"]:
        assert n in names


@pytest.mark.parametrize("variant", ["release", "chaos"])
def test_every_declared_symbol_is_exported(variant):
    # The stress build (pauses in the race windows) exports the same ABI.
    lib = C.load(variant)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert missing == []
    assert lib.dsoar_abi_version() == 2


def test_binding_covers_every_declared_symbol():
    assert declared_functions() <= set(C.SIGNATURES)


def test_version_and_errors():
    lib = C.load()
    assert lib.dsoar_abi_version() == 2
    assert lib.dsoar_error_string(-2).startswith(b"out of memory")
    assert lib.dsoar_error_string(12345) == b"unknown status"


def test_heap_bytes_validates():
    lib = C.load()
    ok = make_desc(4096, 64, [(4, 4, 4)])
    n = lib.dsoar_heap_bytes(ctypes.byref(ok))
    # data: 4096 blocks x 3 arrays x 256 B; plus bitmaps, scan arrays, counters.
    assert n >= 4096 * 768 + 4096 * 12
    for bad in [make_desc(0, 64, [(4,)]), make_desc(16, 48, [(4,)]), make_desc(16, 64, [(3,)]),
                make_desc(16, 64, [])]:
        assert lib.dsoar_heap_bytes(ctypes.byref(bad)) == 0
    # 2^26 blocks: slot 63 of the last block would have the NULL handle.
    assert lib.dsoar_heap_bytes(ctypes.byref(make_desc(1 << 26, 64, [(4,)]))) == 0
    assert lib.dsoar_heap_bytes(ctypes.byref(make_desc((1 << 26) - 1, 64, [(4,)]))) > 0
    h = ctypes.c_void_p()
    assert lib.dsoar_heap_create(ctypes.byref(make_desc(1 << 26, 64, [(4,)])), 256, 1 << 40, None,
                                 ctypes.byref(h)) == C.ERR_INVALID_ARG


def test_create_rejects_bad_buffers():
    lib = C.load()
    d = make_desc(64, 64, [(4,)])
    h = ctypes.c_void_p()
    assert lib.dsoar_heap_create(ctypes.byref(d), None, 1 << 20, None, ctypes.byref(h)) == -1
    assert lib.dsoar_heap_create(ctypes.byref(d), 256, 16, None, ctypes.byref(h)) == -6
    assert lib.dsoar_heap_create(ctypes.byref(d), 257, 1 << 20, None, ctypes.byref(h)) == -1
    assert lib.dsoar_parallel_do(None, 0, 1, None, 0, 0, None) == -1
    assert lib.dsoar_heap_destroy(None) == -1


def test_bitmap_bytes():
    lib = C.load()
    assert lib.dsoar_bitmap_bytes(0, 64) == 0
    assert lib.dsoar_bitmap_bytes(64, 64) == 256 + 256
    assert lib.dsoar_bitmap_bytes(64, 32) == 256 + 256      # two levels of 32-bit containers, padded
    assert lib.dsoar_bitmap_bytes(64, 48) == 0
    assert lib.dsoar_bitmap_bytes(1 << 30, 64) > (1 << 27)
    # 32-bit containers: levels of 2^30, 2^25, 2^20, 2^15, 2^10, 2^5 bits.
    assert lib.dsoar_bitmap_bytes(1 << 30, 32) >= 4 * (2 * sum(-(-(1 << (30 - 5 * k)) // 64) for k in range(6)))


def test_descriptor_width_and_parents_validate():
    lib = C.load()
    ok = [make_desc(4096, 64, [(4, 4)], bitmap_width=w) for w in (0, 32, 64)]
    assert all(lib.dsoar_heap_bytes(ctypes.byref(d)) > 0 for d in ok)
    assert lib.dsoar_heap_bytes(ctypes.byref(make_desc(4096, 64, [(4, 4)], bitmap_width=16))) == 0
    # Subclasses: declared after the parent, starting with its fields.
    good = make_desc(4096, 0, [(4, 8), (4, 8, 4), (4, 8, 4, 4), (4,)], parents=[None, 0, 1, None])
    assert lib.dsoar_heap_bytes(ctypes.byref(good)) > 0
    for types, parents in [([(4, 8), (4, 4, 4)], [None, 0]),      # inherited widths differ
                           ([(4, 8), (4,)], [None, 0]),            # fewer fields than the parent
                           ([(4, 8), (4, 8, 4)], [1, None]),       # parent declared later
                           ([(4, 8), (4, 8, 4)], [0, None])]:      # its own parent
        assert lib.dsoar_heap_bytes(ctypes.byref(make_desc(64, 64, types, parents=parents))) == 0


def test_application_entry_points_validate_without_a_gpu():
    lib = C.load()
    out = ctypes.c_void_p()
    # Sizes: 0 or too large is invalid; otherwise the documented layout.
    assert lib.dsoar_wator_bytes(0) == 0 and lib.dsoar_wator_bytes(1 << 16) == 0
    assert lib.dsoar_wator_bytes(64) == 256 + 64 * 64 + 64 * 64 * 8
    assert lib.dsoar_collide_bytes(0) == 0 and lib.dsoar_collide_bytes((1 << 24) + 1) == 0
    assert lib.dsoar_collide_bytes(100) == 1792 + 1024 + 512
    assert lib.dsoar_traffic_bytes(0, 8) == 0 and lib.dsoar_traffic_bytes(8, 0) == 0
    # A missing heap, handle or rules is an argument error, before any device work.
    wr = C.WatorRules(3, 10, 3, 0, 1)
    assert lib.dsoar_wator_create(None, 64, ctypes.byref(wr), 256, 1 << 20, ctypes.byref(out)) == -1
    assert lib.dsoar_wator_create(None, 64, None, 256, 1 << 20, None) == -1
    cp = C.CollideParams(0.01, 0.01, 0.0, 0)
    assert lib.dsoar_collide_create(None, 16, ctypes.byref(cp), 256, 1 << 20, ctypes.byref(out)) == -1
    tr = C.TrafficRules(5, 0, 0, 0, 1)
    assert lib.dsoar_traffic_create(None, 4, 4, ctypes.byref(tr), 256, 1 << 20, ctypes.byref(out)) == -1
    for fn in ("dsoar_wator_destroy", "dsoar_collide_destroy", "dsoar_traffic_destroy"):
        assert getattr(lib, fn)(None) == -1
    assert lib.dsoar_wator_step(None, 1, 0, None) == -1
    assert lib.dsoar_collide_step(None, 1, 0, None) == -1
    assert lib.dsoar_traffic_step(None, 1, 0, None) == -1
    assert lib.dsoar_wator_read(None, None, None, None, None) == -1
    assert lib.dsoar_wator_init(None, None, None, None, 0, None) == -1
    assert lib.dsoar_heap_set_type_policy(None, 0, C.POLICY_FRESH) == -1


def test_sugarscape_rejects_sugar_beyond_one_byte():
    # A cell keeps its sugar and capacity in seven bits beside the occupancy
    # bit: the wrapper refuses larger inputs before any device work.
    from paper_1809_07444_amd import apps
    from synth import workloads as W
    inp = W.sugar_inputs(16, 8, seed=5)
    for name in ("sugar", "cap"):
        bad = dataclasses.replace(inp, **{name: np.full_like(getattr(inp, name), apps.SUGAR_MAX + 1)})
        with pytest.raises(ValueError):
            apps.Sugarscape(bad, W.SUGAR_RULES)
