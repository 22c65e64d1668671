"""Python view of one device-resident index.  PyTorch supplies device memory
and the current HIP stream; every step runs in libpi's kernels."""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check

_POLICY = {"threshold": _lib.PI_REBUILD_THRESHOLD, "never": _lib.PI_REBUILD_NEVER,
           "always": _lib.PI_REBUILD_ALWAYS, "background": _lib.PI_REBUILD_BACKGROUND,
           "slices": _lib.PI_REBUILD_SLICES}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def to_device_u64(a, device="cuda"):
    """numpy uint64 (or int) array -> int64 CUDA tensor holding the same bits."""
    if isinstance(a, torch.Tensor):
        assert a.dtype in (torch.int64, torch.uint64)
        return a.to(device).view(torch.int64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(device)


def to_device_u8(a, device="cuda"):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.uint8).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8)).to(device)


def to_numpy_u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


class Index:
    """A skip-list index resident on one GPU (C handle from pi_create)."""

    def __init__(self, device: int = 0, max_height: int = 24, log2_inv_p: int = 1,
                 height_seed: int = 0x9E3779B97F4A7C15, rebuild_fraction: float = 0.15,
                 rebuild_policy: str = "threshold", capacity_hint: int = 0, lds_levels: int = 0,
                 profile: int = 0, queries_per_lane: int = 0, blocks_per_cu: int = 0, lds_budget: int = 0,
                 descent_block: int = 0, graph_max_log2: int = 0, small_batch_log2: int = 0,
                 rebuild_min: int = 4096, compact_percent: int = 0, check_writers: int = 0, post_form: int = 0,
                 order_bits: int = 0):
        self._L = _lib.lib()
        cfg = _lib.pi_config()
        check(self._L.pi_config_default(ctypes.byref(cfg)))
        cfg.device = device
        cfg.max_height = max_height
        cfg.log2_inv_p = log2_inv_p
        cfg.height_seed = height_seed
        cfg.rebuild_fraction = rebuild_fraction
        cfg.rebuild_policy = _POLICY[rebuild_policy]
        cfg.capacity_hint = capacity_hint
        cfg.lds_levels = lds_levels
        cfg.profile = profile
        cfg.queries_per_lane = queries_per_lane
        cfg.blocks_per_cu = blocks_per_cu
        cfg.lds_budget = lds_budget
        cfg.descent_block = descent_block
        cfg.graph_max_log2 = graph_max_log2
        cfg.small_batch_log2 = small_batch_log2
        cfg.rebuild_min = rebuild_min
        cfg.compact_percent = compact_percent
        cfg.check_writers = check_writers
        cfg.post_form = post_form
        cfg.order_bits = order_bits
        h = ctypes.c_void_p()
        check(self._L.pi_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", device)

    # ---- lifecycle
    def close(self):
        if getattr(self, "_h", None):
            self._L.pi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        return check(st, self._h)

    # ---- operations
    def bulk_load(self, keys, values, stream=None):
        k = to_device_u64(keys, self.device)
        v = to_device_u64(values, self.device)
        assert k.numel() == v.numel()
        self._check(self._L.pi_bulk_load(self._h, _ptr(k), _ptr(v), k.numel(), _stream(stream)))

    def execute(self, ops, keys, values=None, out_values=None, out_status=None, stream=None):
        """Answers one batch; returns (values int64-bits tensor, status uint8 tensor)."""
        o = to_device_u8(ops, self.device)
        k = to_device_u64(keys, self.device)
        n = k.numel()
        v = to_device_u64(values, self.device) if values is not None else torch.zeros(
            n, dtype=torch.int64, device=self.device)
        assert o.numel() == n and v.numel() == n
        if out_values is None:
            out_values = torch.empty(n, dtype=torch.int64, device=self.device)
        if out_status is None:
            out_status = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._check(self._L.pi_execute_batch(self._h, _ptr(o), _ptr(k), _ptr(v), n, _ptr(out_values),
                                             _ptr(out_status), _stream(stream)))
        return out_values, out_status

    def execute_raw(self, ops_t, keys_t, vals_t, out_v, out_s, stream=None):
        """No conversions: all arguments are device tensors already."""
        self._check(self._L.pi_execute_batch(self._h, _ptr(ops_t), _ptr(keys_t), _ptr(vals_t),
                                             keys_t.numel(), _ptr(out_v), _ptr(out_s), _stream(stream)))

    def execute_noalloc(self, ops_t, keys_t, vals_t, out_v, out_s, stream=None):
        """pi_execute_batch_noalloc: device tensors only; the call allocates
        nothing (its buffers live in the library's per-GPU scratch)."""
        self._check(self._L.pi_execute_batch_noalloc(self._h, _ptr(ops_t), _ptr(keys_t), _ptr(vals_t),
                                                     keys_t.numel(), _ptr(out_v), _ptr(out_s), _stream(stream)))

    def repair(self, stream=None):
        self._check(self._L.pi_repair(self._h, _stream(stream)))

    def export(self, stream=None):
        n = self.stats()["live_nodes"]
        k = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        v = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        got = ctypes.c_uint64()
        self._check(self._L.pi_export(self._h, _ptr(k), _ptr(v), n, ctypes.byref(got), _stream(stream)))
        return k[:got.value], v[:got.value]

    def serve(self, arrival_us, ops, keys, values, deadline_us=100.0, max_batch=0, max_inflight=1, stream=None):
        """Continuous batching of an arrival schedule (pi_serve).  Returns
        (values, status, done_us, batch_ends): device answers, host
        completion time per query and the end index of every micro-batch."""
        arr = np.ascontiguousarray(arrival_us, dtype=np.float64)
        o = to_device_u8(ops, self.device)
        k = to_device_u64(keys, self.device)
        v = to_device_u64(values, self.device)
        n = k.numel()
        assert arr.size == n and o.numel() == n and v.numel() == n
        out_v = torch.empty(n, dtype=torch.int64, device=self.device)
        out_s = torch.empty(n, dtype=torch.uint8, device=self.device)
        done = np.zeros(n, dtype=np.float64)
        ends = np.zeros(max(n, 1), dtype=np.uint64)
        nb = ctypes.c_uint64()
        cfg = _lib.pi_serve_config()
        check(self._L.pi_serve_config_default(ctypes.byref(cfg)))
        cfg.deadline_us = deadline_us
        cfg.max_batch = max_batch
        cfg.max_inflight = max_inflight
        self._check(self._L.pi_serve(self._h, ctypes.byref(cfg), ctypes.c_void_p(arr.ctypes.data), _ptr(o), _ptr(k),
                                     _ptr(v), n, _ptr(out_v), _ptr(out_s), ctypes.c_void_p(done.ctypes.data),
                                     ctypes.c_void_p(ends.ctypes.data), ctypes.byref(nb), _stream(stream)))
        return out_v, out_s, done, ends[:nb.value].astype(np.int64)

    def range_count(self, lo, hi, stream=None):
        """Output offsets u64[n+1] (int64 tensor) of range searches [lo, hi]."""
        lo = to_device_u64(lo, self.device)
        hi = to_device_u64(hi, self.device)
        assert lo.numel() == hi.numel()
        off = torch.empty(lo.numel() + 1, dtype=torch.int64, device=self.device)
        self._check(self._L.pi_range_count(self._h, _ptr(lo), _ptr(hi), lo.numel(), _ptr(off), _stream(stream)))
        return off

    def range_collect(self, lo, hi, offsets, total, stream=None):
        """Pairs of range searches [lo, hi] at the given offsets (total pairs)."""
        lo = to_device_u64(lo, self.device)
        hi = to_device_u64(hi, self.device)
        k = torch.empty(max(total, 1), dtype=torch.int64, device=self.device)
        v = torch.empty(max(total, 1), dtype=torch.int64, device=self.device)
        self._check(self._L.pi_range_collect(self._h, _ptr(lo), _ptr(hi), lo.numel(), _ptr(offsets), _ptr(k),
                                             _ptr(v), _stream(stream)))
        return k[:total], v[:total]

    def range_search(self, lo, hi, stream=None):
        """(counts, keys, values): every live pair of each range [lo[i], hi[i]],
        concatenated in range order.  Synchronises to size the output."""
        lo = to_device_u64(lo, self.device)  # one device copy for both calls
        hi = to_device_u64(hi, self.device)
        off = self.range_count(lo, hi, stream)
        total = int(off[-1].item())
        k, v = self.range_collect(lo, hi, off, total, stream)
        return off[1:] - off[:-1], k, v

    def stats(self):
        s = _lib.pi_stats()
        self._check(self._L.pi_get_stats(self._h, ctypes.byref(s)))
        d = {f: getattr(s, f) for f, _ in _lib.pi_stats._fields_ if f != "level_size"}
        d["level_size"] = list(s.level_size)
        return d

    def profile(self, reset: bool = False):
        """Stage times accumulated since the last reset (index created with profile=1)."""
        p = _lib.pi_profile()
        self._check(self._L.pi_get_profile(self._h, ctypes.byref(p), 1 if reset else 0))
        return {f: getattr(p, f) for f, _ in _lib.pi_profile._fields_}

    def interceptions(self, keys, stream=None):
        k = to_device_u64(keys, self.device)
        n = k.numel()
        ik = torch.empty(n, dtype=torch.int64, device=self.device)
        hd = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._check(self._L.pi_debug_interceptions(self._h, _ptr(k), n, _ptr(ik), _ptr(hd), _stream(stream)))
        return ik, hd

    def level(self, level: int, stream=None):
        n = self.stats()["level_size"][level] if level < 33 else 0
        k = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        d = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        got = ctypes.c_uint64()
        self._check(self._L.pi_debug_level(self._h, level, _ptr(k), _ptr(d), n, ctypes.byref(got),
                                           _stream(stream)))
        return k[:got.value], d[:got.value]

    def writer_selftest(self, stream=None):
        """(error bits of one writer recording twice, of two writers of one
        node) from the checked mode's detection on a private shadow."""
        a, b = ctypes.c_uint32(), ctypes.c_uint32()
        self._check(self._L.pi_debug_writer_selftest(self._h, ctypes.byref(a), ctypes.byref(b), _stream(stream)))
        return a.value, b.value

    def set_storage_bound(self, used_upper: int):
        """Test hook (pi_debug_set_storage_bound): plants the host's bound on
        the storage slots in use."""
        self._check(self._L.pi_debug_set_storage_bound(self._h, used_upper))

    def sort(self, keys, stream=None):
        k = to_device_u64(keys, self.device)
        n = k.numel()
        sk = torch.empty(n, dtype=torch.int64, device=self.device)
        perm = torch.empty(n, dtype=torch.int32, device=self.device)
        self._check(self._L.pi_debug_sort(self._h, _ptr(k), n, _ptr(sk), _ptr(perm), _stream(stream)))
        return sk, perm


class Group:
    """Many indices, one launch (pi_group_*): runs one batch on each of
    several distinct indices of one device."""

    def __init__(self, fused_max: int = 0, max_indices: int = 0, host_threads: int = 0):
        self._L = _lib.lib()
        cfg = _lib.pi_group_config()
        check(self._L.pi_group_config_default(ctypes.byref(cfg)))
        if fused_max:
            cfg.fused_max = fused_max
        if max_indices:
            cfg.max_indices = max_indices
        if host_threads:
            cfg.host_threads = host_threads
        h = ctypes.c_void_p()
        check(self._L.pi_group_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.pi_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _args(self, indices, batches):
        """batches: per index (ops, keys, values, out_values, out_status)
        device tensors (already converted), or None to skip the index."""
        n = len(indices)
        hs = (ctypes.c_void_p * n)(*[ix._h.value for ix in indices])
        bs = (_lib.pi_batch * n)()
        keep = []
        for i, b in enumerate(batches):
            if b is None:
                bs[i].n = 0
                continue
            o, k, v, ov, os_ = b
            keep.append(b)
            bs[i].d_ops, bs[i].d_keys, bs[i].d_values = o.data_ptr(), k.data_ptr(), v.data_ptr()
            bs[i].n = k.numel()
            bs[i].d_out_values, bs[i].d_out_status = ov.data_ptr(), os_.data_ptr()
        return hs, bs, keep

    def _check(self, st):
        if st != _lib.PI_OK:
            msg = self._L.pi_group_last_error(self._h)
            raise _lib.PiError(st, msg.decode() if msg else "")

    def execute(self, indices, batches, stream=None):
        hs, bs, _keep = self._args(indices, batches)
        self._check(self._L.pi_group_execute(self._h, hs, bs, len(indices), _stream(stream)))

    def autotune(self, indices, batches, stream=None) -> int:
        hs, bs, _keep = self._args(indices, batches)
        out = ctypes.c_uint64()
        self._check(self._L.pi_group_autotune(self._h, hs, bs, len(indices), _stream(stream), ctypes.byref(out)))
        return out.value

    def tuning(self):
        """(fused_max, descent_block, lds_budget) chosen by the last autotune
        (0, 0 for the descent shape when it tried none)."""
        f, b, l = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32()
        self._check(self._L.pi_group_tuning(self._h, ctypes.byref(f), ctypes.byref(b), ctypes.byref(l)))
        return f.value, b.value, l.value
