"""ctypes wrapper around the C Pugh skip-list oracle (test infrastructure).

The semantics it implements (paper Section 3.2 query definitions, Definition 1
node, Definition 2 query, Definition 4 interception) are described at the top
of ``skiplist.c``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

SEARCH, INSERT, DELETE = 0, 1, 2
ABSENT, PRESENT, INVALID = 0, 1, 255

DEFAULT_SEED = 0x9E3779B97F4A7C15
DEFAULT_MAX_HEIGHT = 24
DEFAULT_LOG2_INV_P = 1

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    u64, i32, vp = ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [i32, i32, u64]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_force_height.argtypes = [vp, i32]
    lib.orc_size.restype = u64
    lib.orc_size.argtypes = [vp]
    lib.orc_mix64.restype = u64
    lib.orc_mix64.argtypes = [u64]
    lib.orc_height_rule.restype = i32
    lib.orc_height_rule.argtypes = [u64, u64, i32, i32]
    lib.orc_find.restype = i32
    lib.orc_find.argtypes = [vp, u64, ctypes.POINTER(u64)]
    lib.orc_insert.restype = i32
    lib.orc_insert.argtypes = [vp, u64, u64, ctypes.POINTER(u64)]
    lib.orc_erase.restype = i32
    lib.orc_erase.argtypes = [vp, u64, ctypes.POINTER(u64)]
    lib.orc_execute_batch.restype = i32
    lib.orc_execute_batch.argtypes = [vp, vp, vp, vp, u64, vp, vp]
    lib.orc_execute_batch_timed.restype = i32
    lib.orc_execute_batch_timed.argtypes = [vp, vp, vp, vp, u64, vp, vp, ctypes.POINTER(u64)]
    lib.orc_bulk_load.restype = i32
    lib.orc_bulk_load.argtypes = [vp, vp, vp, u64]
    lib.orc_bulk_load_sorted.restype = i32
    lib.orc_bulk_load_sorted.argtypes = [vp, vp, vp, u64]
    lib.orc_export.restype = u64
    lib.orc_export.argtypes = [vp, vp, vp, u64]
    lib.orc_level_count.restype = u64
    lib.orc_level_count.argtypes = [vp, i32]
    lib.orc_level_keys.restype = u64
    lib.orc_level_keys.argtypes = [vp, i32, vp, u64]
    lib.orc_interception.restype = i32
    lib.orc_interception.argtypes = [vp, u64, ctypes.POINTER(u64)]
    lib.orc_range_batch.restype = u64
    lib.orc_range_batch.argtypes = [vp, vp, vp, u64, vp, vp, vp, u64]
    lib.orc_check.restype = i32
    lib.orc_check.argtypes = [vp]
    lib.orc_debug_plant.restype = i32
    lib.orc_debug_plant.argtypes = [vp, i32]
    lib.orc_debug_restore.argtypes = [vp]
    _lib = lib
    return lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def mix64(z: int) -> int:
    """splitmix64 output finalizer as compiled into the oracle."""
    return int(_load().orc_mix64(z))


def height_rule(key: int, seed: int = DEFAULT_SEED, log2_inv_p: int = DEFAULT_LOG2_INV_P,
                max_height: int = DEFAULT_MAX_HEIGHT) -> int:
    return int(_load().orc_height_rule(key, seed, log2_inv_p, max_height))


class SkipList:
    """Single-threaded Pugh skip list; a batch is applied in arrival order."""

    def __init__(self, max_height=DEFAULT_MAX_HEIGHT, log2_inv_p=DEFAULT_LOG2_INV_P,
                 seed=DEFAULT_SEED):
        self._lib = _load()
        self.max_height = max_height
        self.log2_inv_p = log2_inv_p
        self.seed = seed
        self._h = self._lib.orc_create(max_height, log2_inv_p, seed)
        if not self._h:
            raise ValueError("invalid skip-list parameters")

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return int(self._lib.orc_size(self._h))

    def force_height(self, h: int):
        """Test hook: every later insert gets height h (0 restores the rule)."""
        self._lib.orc_force_height(self._h, h)

    def find(self, k):
        v = ctypes.c_uint64()
        hit = self._lib.orc_find(self._h, k, ctypes.byref(v))
        return (PRESENT, v.value) if hit else (ABSENT, 0)

    def insert(self, k, v):
        old = ctypes.c_uint64()
        r = self._lib.orc_insert(self._h, k, v, ctypes.byref(old))
        if r < 0:
            raise MemoryError
        return (PRESENT, old.value) if r == 1 else (ABSENT, 0)

    def erase(self, k):
        old = ctypes.c_uint64()
        r = self._lib.orc_erase(self._h, k, ctypes.byref(old))
        return (PRESENT, old.value) if r == 1 else (ABSENT, 0)

    def execute_batch(self, ops, keys, vals):
        ops = np.ascontiguousarray(ops, dtype=np.uint8)
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals = np.ascontiguousarray(vals, dtype=np.uint64)
        n = ops.size
        assert keys.size == n and vals.size == n
        out_v = np.zeros(n, dtype=np.uint64)
        out_s = np.zeros(n, dtype=np.uint8)
        r = self._lib.orc_execute_batch(self._h, _ptr(ops), _ptr(keys), _ptr(vals), n,
                                        _ptr(out_v), _ptr(out_s))
        if r != 0:
            raise MemoryError
        return out_v, out_s

    def execute_batch_timed(self, ops, keys, vals):
        """execute_batch, plus the nanoseconds the C loop took (monotonic
        clock read inside the library)."""
        ops = np.ascontiguousarray(ops, dtype=np.uint8)
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals = np.ascontiguousarray(vals, dtype=np.uint64)
        n = ops.size
        out_v = np.zeros(n, dtype=np.uint64)
        out_s = np.zeros(n, dtype=np.uint8)
        ns = ctypes.c_uint64()
        r = self._lib.orc_execute_batch_timed(self._h, _ptr(ops), _ptr(keys), _ptr(vals), n, _ptr(out_v),
                                              _ptr(out_s), ctypes.byref(ns))
        if r != 0:
            raise MemoryError
        return out_v, out_s, int(ns.value)

    def bulk_load(self, keys, vals):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals = np.ascontiguousarray(vals, dtype=np.uint64)
        r = self._lib.orc_bulk_load(self._h, _ptr(keys), _ptr(vals), keys.size)
        if r != 0:
            raise RuntimeError(f"orc_bulk_load failed ({r})")

    def bulk_load_sorted(self, keys, vals):
        """Keys must be strictly increasing (already de-duplicated)."""
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals = np.ascontiguousarray(vals, dtype=np.uint64)
        r = self._lib.orc_bulk_load_sorted(self._h, _ptr(keys), _ptr(vals), keys.size)
        if r != 0:
            raise RuntimeError(f"orc_bulk_load_sorted failed ({r})")

    def export(self):
        n = len(self)
        k = np.zeros(n, dtype=np.uint64)
        v = np.zeros(n, dtype=np.uint64)
        got = self._lib.orc_export(self._h, _ptr(k), _ptr(v), n)
        assert got == n
        return k, v

    def level_count(self, level: int) -> int:
        return int(self._lib.orc_level_count(self._h, level))

    def level_keys(self, level: int):
        n = self.level_count(level)
        out = np.zeros(n, dtype=np.uint64)
        got = self._lib.orc_level_keys(self._h, level, _ptr(out), n)
        assert got == n
        return out

    def interception(self, q: int):
        """Key of the interception of q (Definition 4), or None for the head."""
        k = ctypes.c_uint64()
        hit = self._lib.orc_interception(self._h, q, ctypes.byref(k))
        return k.value if hit else None

    def range_batch(self, lo, hi):
        """Range searches [lo[i], hi[i]]: (counts, keys, values), the results
        of all ranges concatenated in range order, each in key order."""
        lo = np.ascontiguousarray(lo, dtype=np.uint64)
        hi = np.ascontiguousarray(hi, dtype=np.uint64)
        assert lo.shape == hi.shape
        counts = np.zeros(lo.size, dtype=np.uint64)
        total = self._lib.orc_range_batch(self._h, _ptr(lo), _ptr(hi), lo.size, _ptr(counts), None, None, 0)
        keys = np.zeros(total, dtype=np.uint64)
        vals = np.zeros(total, dtype=np.uint64)
        got = self._lib.orc_range_batch(self._h, _ptr(lo), _ptr(hi), lo.size, _ptr(counts), _ptr(keys), _ptr(vals),
                                      total)
        assert got == total
        return counts, keys, vals

    def check(self) -> int:
        return int(self._lib.orc_check(self._h))

    def plant(self, kind: int) -> int:
        """Test hook: plants a structural fault (see orc_debug_plant)."""
        return int(self._lib.orc_debug_plant(self._h, kind))

    def restore(self):
        """Test hook: undoes the planted fault."""
        self._lib.orc_debug_restore(self._h)
