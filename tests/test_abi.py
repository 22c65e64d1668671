"""CPU checks of the C ABI: the library loads, exports every entry point that
include/pi.h declares, and its structs have the layout the binding assumes.
No compute call is made (no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1601_00159_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pi.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pi_status|const char \*)\s*(pi_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pi_create", "pi_bulk_load", "pi_execute_batch", "pi_destroy", "pi_export"):
        assert required in names
    assert sorted(_lib.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpi.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "pi.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(pi_config), sizeof(pi_stats),'
                   ' offsetof(pi_config, capacity_hint), offsetof(pi_stats, level_size),'
                   ' sizeof(pi_serve_config), offsetof(pi_serve_config, max_batch));'
                   'printf("%zu %zu\\n", sizeof(pi_group_config), offsetof(pi_group_config, host_threads));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(_lib.pi_config)
    assert int(out[1]) == ctypes.sizeof(_lib.pi_stats)
    assert int(out[2]) == _lib.pi_config.capacity_hint.offset
    assert int(out[3]) == _lib.pi_stats.level_size.offset
    assert int(out[4]) == ctypes.sizeof(_lib.pi_serve_config)
    assert int(out[5]) == _lib.pi_serve_config.max_batch.offset
    assert int(out[6]) == ctypes.sizeof(_lib.pi_group_config)
    assert int(out[7]) == _lib.pi_group_config.host_threads.offset


def test_config_default_without_gpu():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpi.so not built")
    L = _lib.load()
    cfg = _lib.pi_config()
    assert L.pi_config_default(ctypes.byref(cfg)) == _lib.PI_OK
    assert cfg.struct_size == ctypes.sizeof(_lib.pi_config)
    assert cfg.max_height == 24 and cfg.log2_inv_p == 1
    assert cfg.height_seed == 0x9E3779B97F4A7C15
    assert abs(cfg.rebuild_fraction - 0.15) < 1e-7
    assert L.pi_config_default(None) == _lib.PI_ERR_INVALID_ARG
    # NULL handles are rejected before any device work
    assert L.pi_execute_batch(None, None, None, None, 0, None, None, None) == _lib.PI_ERR_INVALID_ARG
    assert L.pi_destroy(None) == _lib.PI_OK
    scfg = _lib.pi_serve_config()
    assert L.pi_serve_config_default(ctypes.byref(scfg)) == _lib.PI_OK
    assert scfg.struct_size == ctypes.sizeof(_lib.pi_serve_config)
    assert scfg.deadline_us == 100.0 and scfg.max_inflight == 1 and scfg.max_batch == 0


@pytest.mark.parametrize("field,value", [("host_threads", 5), ("reserved", 1), ("fused_max", 1 << 31),
                                         ("struct_size", 8)])
def test_group_create_rejects_bad_config_before_device_work(field, value):
    """The group's range checks run before its first device call."""
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpi.so not built")
    L = _lib.load()
    cfg = _lib.pi_group_config()
    assert L.pi_group_config_default(ctypes.byref(cfg)) == _lib.PI_OK
    assert cfg.struct_size == ctypes.sizeof(_lib.pi_group_config)
    assert (cfg.max_indices, cfg.fused_max, cfg.host_threads, cfg.reserved) == (4096, 4096, 4, 0)
    setattr(cfg, field, value)
    h = ctypes.c_void_p(1)
    assert L.pi_group_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.PI_ERR_INVALID_ARG
    assert not h.value


@pytest.mark.parametrize("field,value", [("compact_percent", 1001), ("lds_budget", 13001), ("descent_block", 300),
                                         ("queries_per_lane", 3), ("small_batch_log2", 13), ("graph_max_log2", 11),
                                         ("max_height", 1), ("log2_inv_p", 9), ("rebuild_policy", 5),
                                         ("check_writers", 2), ("post_form", 3),
                                         ("order_bits", 20)])
def test_create_rejects_bad_config_before_device_work(field, value):
    """Every range check of pi_config runs before any device call: on this
    GPU-less host the error names the field, not the missing device."""
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpi.so not built")
    L = _lib.load()
    cfg = _lib.pi_config()
    assert L.pi_config_default(ctypes.byref(cfg)) == _lib.PI_OK
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    assert L.pi_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.PI_ERR_INVALID_ARG
    assert not h.value
    assert b"invalid pi_config field" in L.pi_last_error(None)
