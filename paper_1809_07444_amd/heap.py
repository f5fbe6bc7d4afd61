"""Python binding of the object heap: torch supplies the device buffer and the
stream; every operation is a call into libdsoar.so."""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from . import _capi as C


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def make_desc(num_blocks: int, capacity: int, types: Sequence[Sequence[int]], bitmap_width: int = 64,
              parents: Sequence[int | None] | None = None) -> C.HeapDesc:
    """Heap description: per type the byte width of every field; parents[t]
    is the index of type t's parent type (None: no parent)."""
    if len(types) > C.MAX_TYPES:
        raise ValueError("too many types")
    d = C.HeapDesc()
    d.num_blocks = num_blocks
    d.block_capacity = capacity
    d.num_types = len(types)
    d.bitmap_width = bitmap_width
    for t, fields in enumerate(types):
        if len(fields) > C.MAX_FIELDS:
            raise ValueError("too many fields")
        d.types[t].num_fields = len(fields)
        for f, b in enumerate(fields):
            d.types[t].field_bytes[f] = b
        p = parents[t] if parents is not None else None
        d.types[t].parent = 0 if p is None else p + 1
    return d


def heap_bytes(num_blocks: int, capacity: int, types) -> int:
    return int(C.load().dsoar_heap_bytes(ctypes.byref(make_desc(num_blocks, capacity, types))))


class Heap:
    """A device heap of `num_blocks` blocks with `capacity` slots each.

    `types` lists, per type, the byte width (4 or 8) of every field."""

    def __init__(self, num_blocks: int, capacity: int = 64, types=((4, 4, 4),), device="cuda",
                 stream=None, bitmap_width: int = 64, parents=None):
        self.lib = C.load()
        self.desc = make_desc(num_blocks, capacity, types, bitmap_width, parents)
        self.bitmap_width = bitmap_width
        self.types = [tuple(t) for t in types]
        self.num_blocks, self.capacity = num_blocks, capacity
        nbytes = int(self.lib.dsoar_heap_bytes(ctypes.byref(self.desc)))
        if nbytes == 0:
            raise ValueError("invalid heap description")
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        h = ctypes.c_void_p()
        C.check(self.lib.dsoar_heap_create(ctypes.byref(self.desc), self.buffer.data_ptr(), nbytes,
                                           self._s(), ctypes.byref(h)), "dsoar_heap_create")
        self.h = h

    def _s(self) -> int:
        return _stream_ptr(self.stream)

    def close(self):
        if getattr(self, "h", None):
            self.lib.dsoar_heap_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- control
    def reset(self):
        C.check(self.lib.dsoar_heap_reset(self.h, self._s()), "dsoar_heap_reset")

    def set_launch(self, wg_threads: int, wgs_per_cu: int):
        C.check(self.lib.dsoar_heap_set_launch(self.h, wg_threads, wgs_per_cu), "dsoar_heap_set_launch")

    def set_policy(self, bulk_min: int):
        C.check(self.lib.dsoar_heap_set_policy(self.h, bulk_min), "dsoar_heap_set_policy")

    def set_type_policy(self, type_id: int, policy: int):
        C.check(self.lib.dsoar_heap_set_type_policy(self.h, type_id, policy), "dsoar_heap_set_type_policy")

    def set_search(self, policy: int):
        C.check(self.lib.dsoar_heap_set_search(self.h, policy), "dsoar_heap_set_search")

    def set_reclaim(self, online: bool):
        """Free emptied blocks at the delete that empties them (online) or at enumeration."""
        C.check(self.lib.dsoar_heap_set_reclaim(self.h, 1 if online else 0), "dsoar_heap_set_reclaim")

    def set_unroll(self, blocks_per_pass: int):
        """Blocks per wavefront pass of split do-all methods (1, 2, 4, 8)."""
        C.check(self.lib.dsoar_heap_set_unroll(self.h, blocks_per_pass), "dsoar_heap_set_unroll")

    def set_timing(self, enable: bool):
        C.check(self.lib.dsoar_heap_set_timing(self.h, 1 if enable else 0), "dsoar_heap_set_timing")

    def timing(self) -> dict:
        """{kind name: (launches, total ms)} since the last report."""
        import numpy as np
        kinds = np.zeros(64, np.uint32)
        counts = np.zeros(64, np.uint32)
        ms = np.zeros(64, np.float64)
        n = ctypes.c_uint32()
        C.check(self.lib.dsoar_heap_timing(self.h, kinds.ctypes.data, counts.ctypes.data, ms.ctypes.data, 64,
                                           ctypes.byref(n)), "dsoar_heap_timing")
        return {C.KIND_NAMES.get(int(kinds[i]), str(int(kinds[i]))): (int(counts[i]), float(ms[i]))
                for i in range(n.value)}

    @property
    def type_capacity(self) -> list:
        """Slots per block of each type (the byte-size rule when capacity is 0)."""
        L = self.layout()
        return list(L.type_capacity[:len(self.types)])

    def layout(self) -> C.HeapLayout:
        L = C.HeapLayout()
        C.check(self.lib.dsoar_heap_get_layout(self.h, ctypes.byref(L)), "dsoar_heap_get_layout")
        return L

    def stats(self, raise_sticky: bool = True) -> dict:
        st = C.Stats()
        rc = self.lib.dsoar_heap_stats(self.h, ctypes.byref(st), self._s())
        if rc not in (C.OK, C.ERR_OOM, C.ERR_RETRY_LIMIT, C.ERR_DOUBLE_FREE) or (raise_sticky and rc != C.OK):
            raise C.DsoarError(rc, "dsoar_heap_stats")
        nt = len(self.types)
        return dict(
            allocs=list(st.allocs[:nt]), frees=list(st.frees[:nt]), live=list(st.live_objects[:nt]),
            visits=list(st.visits[:nt]),
            allocated_blocks=list(st.allocated_blocks[:nt]), active_blocks=list(st.active_blocks[:nt]),
            typed_blocks=list(st.typed_blocks[:nt]), reserve_retries=st.reserve_retries,
            slow_paths=st.slow_paths, find_fails=st.find_fails, method_atomics=st.method_atomics,
            online_releases=st.online_releases, blocks_taken=st.blocks_taken,
            blocks_returned=st.blocks_returned, free_blocks=st.free_blocks,
            num_blocks=st.num_blocks, oom=st.oom, retry_limit_hit=st.retry_limit_hit,
            double_free=st.double_free, status=rc)

    def check(self) -> dict:
        v = (ctypes.c_uint32 * 8)()
        rc = self.lib.dsoar_heap_check(self.h, v, self._s())
        if rc not in (C.OK, C.ERR_OOM, C.ERR_RETRY_LIMIT, C.ERR_DOUBLE_FREE):
            raise C.DsoarError(rc, "dsoar_heap_check")
        out = {name: int(v[i]) for i, name in enumerate(C.INV_NAMES) if v[i]}
        if rc != C.OK:
            out["sticky"] = C.ERRORS[rc]
        return out

    # ---------------------------------------------------------- do-all etc
    def enumerate(self, t: int):
        C.check(self.lib.dsoar_enumerate(self.h, t, self._s()), "dsoar_enumerate")

    def enum_count(self, t: int) -> int:
        c = ctypes.c_uint32()
        C.check(self.lib.dsoar_enum_count(self.h, t, ctypes.byref(c), self._s()), "dsoar_enum_count")
        return int(c.value)

    def enum_arrays(self, t: int, count: int):
        """(R, S) of the last enumeration as torch views (R int32 ids, S int64 snapshots)."""
        r, s = ctypes.c_uint64(), ctypes.c_uint64()
        C.check(self.lib.dsoar_enum_arrays(self.h, t, ctypes.byref(r), ctypes.byref(s)), "dsoar_enum_arrays")
        base = self.buffer.data_ptr()
        R = self.buffer[r.value - base: r.value - base + 4 * count].view(torch.int32)
        S = self.buffer[s.value - base: s.value - base + 8 * count].view(torch.int64)
        return R, S

    def reclaim(self):
        C.check(self.lib.dsoar_reclaim(self.h, self._s()), "dsoar_reclaim")

    def parallel_do(self, t: int, method: int, args=None, flags: int = C.DO_PERSISTENT):
        if args is None:
            ptr, n = None, 0
        else:
            ptr, n = ctypes.byref(args), ctypes.sizeof(args)
        C.check(self.lib.dsoar_parallel_do(self.h, t, method, ptr, n, flags, self._s()), "dsoar_parallel_do")

    def visit_counts(self, t: int, flags: int = C.DO_PERSISTENT) -> torch.Tensor:
        counts = torch.zeros(self.num_blocks * 64, dtype=torch.int32, device=self.buffer.device)
        self.parallel_do(t, C.METHOD_VISIT_COUNT, C.VisitArgs(counts.data_ptr()), flags)
        return counts

    def delete_if_mod(self, t: int, field: int, modulus: int, residue: int, flags: int = C.DO_PERSISTENT):
        self.parallel_do(t, C.METHOD_DELETE_IF_MOD, C.ModArgs(field, modulus, residue), flags)

    def gather(self, t: int, key_field: int, field: int, num_keys: int, flags: int = C.DO_PERSISTENT):
        wide = self.types[t][field] == 8
        out = torch.zeros(max(num_keys, 1), dtype=torch.int64 if wide else torch.int32, device=self.buffer.device)
        present = torch.zeros(max(num_keys, 1), dtype=torch.uint8, device=self.buffer.device)
        a = C.GatherArgs(key_field, field, num_keys, 0, out.data_ptr(), present.data_ptr())
        self.parallel_do(t, C.METHOD_FIELD_GATHER, a, flags)
        return out[:num_keys], present[:num_keys]

    # -------------------------------------------------------- alloc / free
    def alloc_n(self, t: int, n: int) -> torch.Tensor:
        out = torch.empty(max(n, 1), dtype=torch.int32, device=self.buffer.device)
        C.check(self.lib.dsoar_alloc_n(self.h, t, n, out.data_ptr(), self._s()), "dsoar_alloc_n")
        return out[:n]

    def stress_churn(self, n: int, rounds: int, keep: int, seed: int = 1, spread: int = 1):
        """Runs the new/delete stress kernel; returns (kept handles [n, rounds], error count)."""
        out = torch.empty(n * rounds, dtype=torch.int32, device=self.buffer.device)
        err = torch.zeros(1, dtype=torch.int32, device=self.buffer.device)
        torch.cuda.synchronize()
        C.check(self.lib.dsoar_stress_churn(self.h, n, rounds, keep, spread, seed, out.data_ptr(), err.data_ptr(),
                                            self._s()),
                "dsoar_stress_churn")
        torch.cuda.synchronize()
        return out.view(n, rounds), int(err.item())

    def free_n(self, objs: torch.Tensor):
        objs = objs.to(torch.int32).contiguous()
        C.check(self.lib.dsoar_free_n(self.h, objs.data_ptr(), objs.numel(), self._s()), "dsoar_free_n")

    def field_read(self, t: int, field: int, objs: torch.Tensor) -> torch.Tensor:
        objs = objs.to(torch.int32).contiguous()
        out = torch.zeros(max(objs.numel(), 1), dtype=torch.int32, device=self.buffer.device)
        C.check(self.lib.dsoar_field_read(self.h, t, field, objs.data_ptr(), objs.numel(), out.data_ptr(),
                                          self._s()), "dsoar_field_read")
        return out[:objs.numel()]

    def field_write(self, t: int, field: int, objs: torch.Tensor, values: torch.Tensor):
        objs = objs.to(torch.int32).contiguous()
        values = values.contiguous()
        assert values.element_size() == 4 and values.numel() == objs.numel()
        C.check(self.lib.dsoar_field_write(self.h, t, field, objs.data_ptr(), objs.numel(), values.data_ptr(),
                                           self._s()), "dsoar_field_write")

    # ------------------------------------------------------- raw inspection
    def raw(self):
        """Views of the heap's bookkeeping arrays in device memory."""
        L = self.layout()
        M = self.num_blocks
        b = self.buffer
        ob = b[L.obj_bitmap_offset: L.obj_bitmap_offset + 8 * M].view(torch.int64)
        tw = b[L.block_type_offset: L.block_type_offset + 4 * M].view(torch.int32)
        t8 = tw & 0xFF
        bt = torch.where(t8 == 0xFF, torch.full_like(t8, -1), t8)  # type, -1 = free
        nbm = 1 + 2 * len(self.types)
        # One row per bitmap, one element per container (int64 or int32 by
        # the heap's bitmap width), indexed by the levels' container offsets.
        cw = L.bitmap_width
        bms = b[L.bitmaps_offset: L.bitmaps_offset + nbm * L.bitmap_stride].view(
            torch.int64 if cw == 64 else torch.int32)
        bms = bms.view(nbm, L.bitmap_stride * 8 // cw)
        levels = [(L.level_word_offset[i], L.level_words[i]) for i in range(L.num_levels)]
        return dict(obj_bitmap=ob, block_type=bt, bitmaps=bms, levels=levels, bitmap_width=cw)


class DeviceBitmap:
    """A stand-alone device hierarchical bitmap (tests of the bitmap operations)."""

    def __init__(self, nbits: int, all_set: bool = False, device="cuda", width: int = 64):
        self.lib = C.load()
        self.nbits = nbits
        self.width = width
        nbytes = int(self.lib.dsoar_bitmap_bytes(nbits, width))
        if nbytes == 0:
            raise ValueError("bad bitmap size")
        self.buffer = torch.empty(nbytes // 8, dtype=torch.int64, device=device)
        C.check(self.lib.dsoar_bitmap_init(self.buffer.data_ptr(), nbits, width, 1 if all_set else 0,
                                           _stream_ptr()), "dsoar_bitmap_init")

    def run(self, ops: torch.Tensor, starts: torch.Tensor | None = None) -> torch.Tensor:
        """ops: int32 [n, 2] (kind, pos) run concurrently, one wavefront each."""
        ops = ops.to(torch.int32).contiguous()
        n = ops.shape[0]
        res = torch.zeros(max(n, 1), dtype=torch.int32, device=self.buffer.device)
        st = None
        if starts is not None:
            starts = starts.to(torch.int32).contiguous()
            st = starts.data_ptr()
        C.check(self.lib.dsoar_bitmap_run(self.buffer.data_ptr(), self.nbits, self.width, ops.data_ptr(), n, st,
                                          res.data_ptr(), _stream_ptr()), "dsoar_bitmap_run")
        return res[:n]

    def level_words(self):
        """Per level, its containers (int64 at width 64, int32 at width 32);
        levels start at 8-byte boundaries, level 0 first."""
        units = self.buffer.view(torch.int32)
        out = []
        n, off = self.nbits, 0
        while True:
            c = -(-n // self.width)
            lv = units[off: off + c * self.width // 32]
            out.append(lv.view(torch.int64) if self.width == 64 else lv)
            off += 2 * (-(-n // 64))
            if n <= self.width:
                break
            n = c
        return out
