"""ctypes binding of libpi (include/pi.h): same names, argument marshalling
only.  Every computation runs in the HIP kernels of libpi.so; there is no
other code path, and importing this module fails if the library was not
built."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpi.so")

PI_OK = 0
PI_ERR_INVALID_ARG = -1
PI_ERR_OUT_OF_MEMORY = -2
PI_ERR_STATE = -3
PI_ERR_DEVICE = -4
PI_ERR_CAPACITY = -5

PI_OP_SEARCH, PI_OP_INSERT, PI_OP_DELETE = 0, 1, 2
PI_R_ABSENT, PI_R_PRESENT, PI_R_INVALID = 0, 1, 255
PI_REBUILD_THRESHOLD, PI_REBUILD_NEVER, PI_REBUILD_ALWAYS, PI_REBUILD_BACKGROUND, PI_REBUILD_SLICES = 0, 1, 2, 3, 4

STATUS_NAMES = {PI_OK: "PI_OK", PI_ERR_INVALID_ARG: "PI_ERR_INVALID_ARG",
                PI_ERR_OUT_OF_MEMORY: "PI_ERR_OUT_OF_MEMORY", PI_ERR_STATE: "PI_ERR_STATE",
                PI_ERR_DEVICE: "PI_ERR_DEVICE", PI_ERR_CAPACITY: "PI_ERR_CAPACITY"}


class pi_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("max_height", ctypes.c_uint32), ("log2_inv_p", ctypes.c_uint32),
                ("height_seed", ctypes.c_uint64), ("rebuild_fraction", ctypes.c_float),
                ("rebuild_policy", ctypes.c_uint32), ("capacity_hint", ctypes.c_uint64),
                ("lds_levels", ctypes.c_uint32), ("profile", ctypes.c_uint32),
                ("queries_per_lane", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("lds_budget", ctypes.c_uint32), ("descent_block", ctypes.c_uint32),
                ("graph_max_log2", ctypes.c_uint32), ("small_batch_log2", ctypes.c_uint32),
                ("compact_percent", ctypes.c_uint32), ("rebuild_min", ctypes.c_uint64),
                ("check_writers", ctypes.c_uint32), ("post_form", ctypes.c_uint32),
                ("order_bits", ctypes.c_uint32)]


class pi_profile(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("rebuilds", ctypes.c_uint64),
                ("sort_ms", ctypes.c_double), ("descend_ms", ctypes.c_double),
                ("own_ms", ctypes.c_double), ("link_ms", ctypes.c_double),
                ("rebuild_ms", ctypes.c_double)]


class pi_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "batches", "queries", "hits", "invalid", "new_nodes", "deletes", "revives", "changes",
        "repairs", "live_nodes", "base_nodes", "overflow_nodes", "capacity")] + [
        ("n_levels", ctypes.c_uint32), ("lds_from", ctypes.c_uint32),
        ("level_size", ctypes.c_uint64 * 33), ("index_rebuilds", ctypes.c_uint64),
        ("slice_rounds", ctypes.c_uint64), ("slices_repaired", ctypes.c_uint64), ("slices", ctypes.c_uint64)]


EXPORTED = ["pi_config_default", "pi_create", "pi_destroy", "pi_bulk_load", "pi_execute_batch",
            "pi_repair", "pi_export", "pi_range_count", "pi_range_collect", "pi_serve_config_default", "pi_serve", "pi_group_config_default", "pi_group_create",
            "pi_group_destroy", "pi_group_execute", "pi_group_autotune", "pi_group_tuning", "pi_group_last_error", "pi_get_stats", "pi_get_profile", "pi_last_error", "pi_debug_interceptions",
            "pi_debug_level", "pi_debug_sort", "pi_debug_set_storage_bound", "pi_debug_writer_selftest",
            "pi_execute_batch_noalloc"]


class pi_serve_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32),
                ("deadline_us", ctypes.c_double), ("max_batch", ctypes.c_uint64)]


class pi_batch(ctypes.Structure):
    _fields_ = [("d_ops", ctypes.c_void_p), ("d_keys", ctypes.c_void_p), ("d_values", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("d_out_values", ctypes.c_void_p), ("d_out_status", ctypes.c_void_p)]


class pi_group_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_indices", ctypes.c_uint32), ("fused_max", ctypes.c_uint64),
                ("host_threads", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class PiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(f"libpi.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
    sig = {
        "pi_config_default": ([ctypes.POINTER(pi_config)], i32),
        "pi_create": ([ctypes.POINTER(pi_config), ctypes.POINTER(vp)], i32),
        "pi_destroy": ([vp], i32),
        "pi_bulk_load": ([vp, vp, vp, u64, vp], i32),
        "pi_execute_batch": ([vp, vp, vp, vp, u64, vp, vp, vp], i32),
        "pi_repair": ([vp, vp], i32),
        "pi_export": ([vp, vp, vp, u64, ctypes.POINTER(u64), vp], i32),
        "pi_range_count": ([vp, vp, vp, u64, vp, vp], i32),
        "pi_range_collect": ([vp, vp, vp, u64, vp, vp, vp, vp], i32),
        "pi_serve_config_default": ([ctypes.POINTER(pi_serve_config)], i32),
        "pi_serve": ([vp, ctypes.POINTER(pi_serve_config), vp, vp, vp, vp, u64, vp, vp, vp, vp,
                      ctypes.POINTER(u64), vp], i32),
        "pi_group_config_default": ([ctypes.POINTER(pi_group_config)], i32),
        "pi_group_create": ([ctypes.POINTER(pi_group_config), ctypes.POINTER(vp)], i32),
        "pi_group_destroy": ([vp], i32),
        "pi_group_execute": ([vp, vp, ctypes.POINTER(pi_batch), u32, vp], i32),
        "pi_group_autotune": ([vp, vp, ctypes.POINTER(pi_batch), u32, vp, ctypes.POINTER(u64)], i32),
        "pi_group_tuning": ([vp, ctypes.POINTER(u64), ctypes.POINTER(u32), ctypes.POINTER(u32)], i32),
        "pi_group_last_error": ([vp], ctypes.c_char_p),
        "pi_get_stats": ([vp, ctypes.POINTER(pi_stats)], i32),
        "pi_get_profile": ([vp, ctypes.POINTER(pi_profile), i32], i32),
        "pi_last_error": ([vp], ctypes.c_char_p),
        "pi_debug_interceptions": ([vp, vp, u64, vp, vp, vp], i32),
        "pi_debug_level": ([vp, u32, vp, vp, u64, ctypes.POINTER(u64), vp], i32),
        "pi_debug_sort": ([vp, vp, u64, vp, vp, vp], i32),
        "pi_debug_set_storage_bound": ([vp, u64], i32),
        "pi_debug_writer_selftest": ([vp, ctypes.POINTER(u32), ctypes.POINTER(u32), vp], i32),
        "pi_execute_batch_noalloc": ([vp, vp, vp, vp, u64, vp, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def check(status, handle=None):
    if status != PI_OK:
        msg = lib().pi_last_error(handle)
        raise PiError(status, msg.decode() if msg else "")
    return status
