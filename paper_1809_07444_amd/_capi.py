"""ctypes declarations of the C ABI in include/dsoar.h (argument marshalling only).

Loading fails loudly when libdsoar.so is missing: there is no fallback path.
The stress tests select libdsoar_chaos.so (the same library built with
pauses in the heap's race windows) with `using("chaos")`."""
from __future__ import annotations

import contextlib
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsoar.so")
LIB_PATHS = {"release": LIB_PATH, "chaos": os.path.join(HERE, "libdsoar_chaos.so")}

MAX_TYPES = 8
MAX_FIELDS = 8
NULL = 0xFFFFFFFF

OK = 0
ERRORS = {
    -1: "DSOAR_ERR_INVALID_ARG", -2: "DSOAR_ERR_OOM", -3: "DSOAR_ERR_RETRY_LIMIT",
    -4: "DSOAR_ERR_HIP", -5: "DSOAR_ERR_DOUBLE_FREE", -6: "DSOAR_ERR_TOO_SMALL",
    -7: "DSOAR_ERR_UNSUPPORTED",
}
ERR_INVALID_ARG, ERR_OOM, ERR_RETRY_LIMIT, ERR_DOUBLE_FREE = -1, -2, -3, -5

DO_PERSISTENT, DO_PLAIN, DO_REUSE_ENUM = 0, 1, 2
GRAPH = GOL_GRAPH = 0x100
POLICY_DENSE, POLICY_FRESH, POLICY_BOUNDED = 0, 1, 2
SEARCH_HASHED, SEARCH_LOWEST, SEARCH_XCD = 0, 1, 2
METHOD_VISIT_COUNT, METHOD_DELETE_IF_MOD, METHOD_MICRO_UPDATE, METHOD_MICRO_CULL, METHOD_FIELD_GATHER = 1, 2, 3, 4, 5
BM_TRY_SET, BM_TRY_CLEAR, BM_SET, BM_CLEAR, BM_TRY_FIND_SET, BM_FIND_CLEAR = range(6)
KIND_NAMES = {1: "enumerate", 10: "visit_count", 11: "delete_if_mod", 12: "gather", 20: "micro_update",
              21: "micro_cull", 30: "gol_alive_prep", 31: "gol_cand_prep", 32: "gol_alive_update",
              33: "gol_cand_update", 35: "gol_update", 40: "sugar_choose", 41: "sugar_move", 42: "sugar_eat",
              43: "sugar_request", 44: "sugar_birth", 34: "gol_delete_world", 45: "sugar_delete_world",
              50: "traffic_decide", 51: "traffic_drive", 60: "collide_force", 61: "collide_move",
              62: "collide_root", 63: "collide_target", 64: "collide_merge", 65: "collide_remove",
              70: "wator_fish_decide", 71: "wator_fish_move", 72: "wator_shark_decide",
              73: "wator_shark_move", 74: "wator_fish_eaten", 75: "wator_fish_read", 76: "wator_shark_read",
              22: "micro_create", 36: "gol_init", 37: "gol_admit", 46: "sugar_regrow", 47: "sugar_admit",
              52: "traffic_entry", 53: "traffic_init", 66: "collide_init",
              77: "wator_init", 78: "wator_tick"}
INV_NAMES = ["bitmap_range", "allocated", "active", "active_implies_allocated", "free",
             "container", "live_count", "free_count"]

u32, u64, i32, vp, sz = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t


class TypeLayout(ctypes.Structure):
    _fields_ = [("num_fields", u32), ("field_bytes", u32 * MAX_FIELDS), ("parent", u32)]


class HeapDesc(ctypes.Structure):
    _fields_ = [("num_blocks", u32), ("block_capacity", u32), ("num_types", u32), ("bitmap_width", u32),
                ("types", TypeLayout * MAX_TYPES)]


class HeapLayout(ctypes.Structure):
    _fields_ = [("total_bytes", u64), ("data_offset", u64), ("block_stride", u64),
                ("obj_bitmap_offset", u64), ("block_type_offset", u64), ("bitmaps_offset", u64),
                ("bitmap_stride", u64), ("bitmap_width", u32), ("num_levels", u32), ("level_word_offset", u32 * 8),
                ("level_words", u32 * 8), ("field_offset", (u32 * MAX_FIELDS) * MAX_TYPES),
                ("type_capacity", u32 * MAX_TYPES)]


class Stats(ctypes.Structure):
    _fields_ = [("allocs", u64 * MAX_TYPES), ("frees", u64 * MAX_TYPES), ("live_objects", u64 * MAX_TYPES),
                ("visits", u64 * MAX_TYPES),
                ("allocated_blocks", u32 * MAX_TYPES), ("active_blocks", u32 * MAX_TYPES),
                ("typed_blocks", u32 * MAX_TYPES), ("reserve_retries", u64), ("slow_paths", u64),
                ("find_fails", u64), ("method_atomics", u64), ("online_releases", u64), ("blocks_taken", u64),
                ("blocks_returned", u64), ("free_blocks", u32), ("num_blocks", u32), ("oom", u32),
                ("retry_limit_hit", u32), ("double_free", u32), ("reserved", u32)]


class CollideParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("eps2", ctypes.c_float), ("r2_merge", ctypes.c_float), ("reserved", u32)]


class TrafficRules(ctypes.Structure):
    _fields_ = [("vmax", i32), ("p_slow24", u32), ("p_in24", u32), ("reserved", u32), ("seed", u64)]


class WatorRules(ctypes.Structure):
    _fields_ = [("fish_breed", i32), ("shark_breed", i32), ("starve", i32), ("reserved", u32), ("seed", u64)]


class SugarRules(ctypes.Structure):
    _fields_ = [("max_age", i32), ("repro_min", i32), ("fertile_min", i32), ("fertile_max", i32),
                ("seed", u64)]


class VisitArgs(ctypes.Structure):
    _fields_ = [("counts_dev", vp)]


class ModArgs(ctypes.Structure):
    _fields_ = [("field", u32), ("modulus", i32), ("residue", i32)]


class GatherArgs(ctypes.Structure):
    _fields_ = [("key_field", u32), ("field", u32), ("num_keys", u32), ("reserved", u32),
                ("out_dev", vp), ("present_dev", vp)]


H = vp  # dsoar_heap*

SIGNATURES = {
    "dsoar_heap_bytes": (sz, [ctypes.POINTER(HeapDesc)]),
    "dsoar_heap_create": (ctypes.c_int, [ctypes.POINTER(HeapDesc), vp, sz, vp, ctypes.POINTER(vp)]),
    "dsoar_heap_destroy": (ctypes.c_int, [H]),
    "dsoar_heap_reset": (ctypes.c_int, [H, vp]),
    "dsoar_heap_get_layout": (ctypes.c_int, [H, ctypes.POINTER(HeapLayout)]),
    "dsoar_heap_set_launch": (ctypes.c_int, [H, u32, u32]),
    "dsoar_heap_set_policy": (ctypes.c_int, [H, u32]),
    "dsoar_heap_set_type_policy": (ctypes.c_int, [H, u32, u32]),
    "dsoar_heap_set_unroll": (ctypes.c_int, [H, u32]),
    "dsoar_heap_set_reclaim": (ctypes.c_int, [H, ctypes.c_int]),
    "dsoar_heap_set_search": (ctypes.c_int, [H, u32]),
    "dsoar_stress_churn": (ctypes.c_int, [H, u32, u32, u32, u32, u32, vp, vp, vp]),
    "dsoar_last_hip_error": (ctypes.c_int, [H]),
    "dsoar_heap_set_timing": (ctypes.c_int, [H, ctypes.c_int]),
    "dsoar_heap_timing": (ctypes.c_int, [H, vp, vp, vp, u32, ctypes.POINTER(u32)]),
    "dsoar_enumerate": (ctypes.c_int, [H, u32, vp]),
    "dsoar_enumerate_noalloc": (ctypes.c_int, [H, u32, vp, vp, vp, vp]),
    "dsoar_enum_count": (ctypes.c_int, [H, u32, ctypes.POINTER(u32), vp]),
    "dsoar_enum_arrays": (ctypes.c_int, [H, u32, ctypes.POINTER(u64), ctypes.POINTER(u64)]),
    "dsoar_reclaim": (ctypes.c_int, [H, vp]),
    "dsoar_parallel_do": (ctypes.c_int, [H, u32, u32, vp, sz, u32, vp]),
    "dsoar_heap_stats": (ctypes.c_int, [H, ctypes.POINTER(Stats), vp]),
    "dsoar_heap_check": (ctypes.c_int, [H, ctypes.POINTER(u32), vp]),
    "dsoar_alloc_n": (ctypes.c_int, [H, u32, u32, vp, vp]),
    "dsoar_free_n": (ctypes.c_int, [H, vp, u32, vp]),
    "dsoar_field_read": (ctypes.c_int, [H, u32, u32, vp, u32, vp, vp]),
    "dsoar_field_write": (ctypes.c_int, [H, u32, u32, vp, u32, vp, vp]),
    "dsoar_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "dsoar_abi_version": (ctypes.c_int, []),
    "dsoar_bitmap_bytes": (sz, [u32, u32]),
    "dsoar_bitmap_init": (ctypes.c_int, [vp, u32, u32, ctypes.c_int, vp]),
    "dsoar_bitmap_run": (ctypes.c_int, [vp, u32, u32, vp, u32, vp, vp, vp]),
    "dsoar_micro_init": (ctypes.c_int, [H, u32, u32, vp, vp, vp]),
    "dsoar_micro_step": (ctypes.c_int, [H, u32, u32, vp, vp, u32, vp]),
    "dsoar_probe_atomics": (ctypes.c_int, [vp, u32, u32, u32, u32, vp]),
    "dsoar_probe_copy": (ctypes.c_int, [vp, vp, sz, vp]),
    "dsoar_gol_bytes": (sz, [u32, vp]),
    "dsoar_gol_create": (ctypes.c_int, [H, u32, vp, vp, sz, vp, ctypes.POINTER(vp)]),
    "dsoar_gol_destroy": (ctypes.c_int, [vp]),
    "dsoar_gol_init": (ctypes.c_int, [vp, vp, vp]),
    "dsoar_gol_step": (ctypes.c_int, [vp, u32, u32, vp]),
    "dsoar_gol_read": (ctypes.c_int, [vp, vp, vp]),
    "dsoar_gol_total_cells": (u32, [vp]),
    "dsoar_golpool_bytes": (sz, [u32, u32]),
    "dsoar_golpool_create": (ctypes.c_int, [H, u32, u32, vp, sz, vp, ctypes.POINTER(vp)]),
    "dsoar_gol_admit": (ctypes.c_int, [vp, u32, u32, u32, vp, vp]),
    "dsoar_gol_retire": (ctypes.c_int, [vp, u32, vp]),
    "dsoar_gol_read_world": (ctypes.c_int, [vp, u32, vp, vp]),
    "dsoar_sugarpool_bytes": (sz, [u32, u32]),
    "dsoar_sugarpool_create": (ctypes.c_int, [H, u32, u32, vp, vp, sz, ctypes.POINTER(vp)]),
    "dsoar_sugar_admit": (ctypes.c_int, [vp, u32, u32, u32, u64, u32, vp, vp, vp, vp, vp, vp, vp, vp]),
    "dsoar_sugar_retire": (ctypes.c_int, [vp, u32, vp]),
    "dsoar_sugar_read_world": (ctypes.c_int, [vp, u32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(u64), vp]),
    "dsoar_sugar_bytes": (sz, [u32]),
    "dsoar_sugar_create": (ctypes.c_int, [H, u32, vp, vp, sz, ctypes.POINTER(vp)]),
    "dsoar_sugar_destroy": (ctypes.c_int, [vp]),
    "dsoar_sugar_init": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, u32, vp]),
    "dsoar_sugar_step": (ctypes.c_int, [vp, u32, u32, vp]),
    "dsoar_sugar_read": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(u32), vp]),
    "dsoar_collide_bytes": (sz, [u32]),
    "dsoar_collide_create": (ctypes.c_int, [H, u32, vp, vp, sz, ctypes.POINTER(vp)]),
    "dsoar_collide_destroy": (ctypes.c_int, [vp]),
    "dsoar_collide_init": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
    "dsoar_collide_step": (ctypes.c_int, [vp, u32, u32, vp]),
    "dsoar_collide_read": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
    "dsoar_traffic_bytes": (sz, [u32, u32]),
    "dsoar_traffic_create": (ctypes.c_int, [H, u32, u32, vp, vp, sz, ctypes.POINTER(vp)]),
    "dsoar_traffic_destroy": (ctypes.c_int, [vp]),
    "dsoar_traffic_init": (ctypes.c_int, [vp, vp, u32, vp]),
    "dsoar_traffic_step": (ctypes.c_int, [vp, u32, u32, vp]),
    "dsoar_traffic_read": (ctypes.c_int, [vp, vp, vp]),
    "dsoar_wator_bytes": (sz, [u32]),
    "dsoar_wator_create": (ctypes.c_int, [H, u32, vp, vp, sz, ctypes.POINTER(vp)]),
    "dsoar_wator_destroy": (ctypes.c_int, [vp]),
    "dsoar_wator_init": (ctypes.c_int, [vp, vp, vp, vp, u32, vp]),
    "dsoar_wator_step": (ctypes.c_int, [vp, u32, u32, vp]),
    "dsoar_wator_read": (ctypes.c_int, [vp, vp, vp, vp, vp]),
}

_libs: dict = {}
_variant = "release"


class DsoarError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {ERRORS.get(code, code)}")


def load(variant: str | None = None) -> ctypes.CDLL:
    """Loads the library of `variant` (default: the one `using` selected,
    else the release build) from the package directory; never builds, never
    falls back."""
    v = variant or _variant
    if v not in _libs:
        path = LIB_PATHS[v]
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with "
                              "`python -m paper_1809_07444_amd.build` (hipcc, gfx950)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _libs[v] = lib
    return _libs[v]


@contextlib.contextmanager
def using(variant: str):
    """Objects created inside the block bind to the library of `variant`."""
    global _variant
    if variant not in LIB_PATHS:
        raise ValueError(variant)
    old, _variant = _variant, variant
    try:
        yield load(variant)
    finally:
        _variant = old


def check(code: int, what: str) -> int:
    if code != OK:
        raise DsoarError(code, what)
    return code
