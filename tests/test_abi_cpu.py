"""CPU-only checks of the C-ABI library: it loads, exports every function
include/rt.h declares, reports status strings, and rejects invalid arguments
before touching a device.  Also checks that the product and the oracle share
no code."""
from __future__ import annotations

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2603_00292_amd import _capi

    if not os.path.exists(_capi.LIB_PATH):
        from paper_2603_00292_amd import build_lib

        build_lib.build()
    return _capi.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), f"{n} declared in rt.h but not exported"
    from paper_2603_00292_amd import _capi

    assert sorted(_capi.EXPORTS) == names


def test_status_strings(lib):
    from paper_2603_00292_amd import _capi as c

    for code, name in [(c.RT_SUCCESS, "RT_SUCCESS"), (c.RT_ERROR_INVALID_VALUE, "RT_ERROR_INVALID_VALUE"),
                       (c.RT_ERROR_OUT_OF_MEMORY, "RT_ERROR_OUT_OF_MEMORY"),
                       (c.RT_ERROR_NO_DEVICE, "RT_ERROR_NO_DEVICE"), (c.RT_ERROR_HIP, "RT_ERROR_HIP"),
                       (c.RT_ERROR_UNSUPPORTED, "RT_ERROR_UNSUPPORTED"),
                       (c.RT_ERROR_INDEX_OUT_OF_RANGE, "RT_ERROR_INDEX_OUT_OF_RANGE"),
                       (c.RT_ERROR_STACK_OVERFLOW, "RT_ERROR_STACK_OVERFLOW")]:
        assert lib.rt_status_string(code).decode() == name
    assert lib.rt_version() == 100


def test_null_arguments_rejected_on_host(lib):
    from paper_2603_00292_amd import _capi as c

    P = C.c_void_p
    h = C.c_void_p()
    assert lib.rt_context_create(0, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_context_destroy(None) == c.RT_ERROR_INVALID_VALUE
    v = c.rt_variant(16, 256)
    assert lib.rt_context_set_variant(None, C.byref(v)) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_context_set_timing(None, 4) == c.RT_ERROR_INVALID_VALUE
    cnt = C.c_uint32(7)
    assert lib.rt_context_read_timing(None, None, 0, C.byref(cnt)) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_build(None, None, 0, None, None, 0, None, None, C.byref(h)) == c.RT_ERROR_INVALID_VALUE
    assert b"NULL context" in lib.rt_last_error_message()
    assert lib.rt_build(None, None, 0, None, None, 0, None, None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_trace_closest(None, None, 0, None, None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_trace_any(None, None, 0, None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_trace_backward(None, None, None, None, 0, None, None, None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_accel_destroy(None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_accel_get_info(None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_batch_plan_create(None, None, None, None, None, 0, C.byref(h)) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_batch_plan_launch(None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_batch_plan_graph(None, None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_batch_plan_destroy(None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_update_instances(None, None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_accel_set_instance_masks(None, None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_refit(None, None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_trace_all(None, None, 0, None, 1, None, None, None, None) == c.RT_ERROR_INVALID_VALUE
    assert lib.rt_trace_counters(None, None, 0, 0, None, None, None, None) == c.RT_ERROR_INVALID_VALUE
    for k in (0, 5, 16):
        assert lib.rt_trace_counters_ex(None, None, 0, 0, None, None, None, k, None) == c.RT_ERROR_INVALID_VALUE
        assert b"n_counters" in lib.rt_last_error_message()
    del P


def test_no_device_reported(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2603_00292_amd import _capi as c

    h = C.c_void_p()
    assert lib.rt_context_create(0, C.byref(h)) == c.RT_ERROR_NO_DEVICE
    assert h.value is None


def _sources(d, exts):
    for dp, _, fs in os.walk(os.path.join(ROOT, d)):
        if "_build" in dp or "__pycache__" in dp:
            continue
        for f in fs:
            if f.endswith(exts):
                yield os.path.join(dp, f)


def test_product_and_oracle_share_no_code():
    for p in _sources("paper_2603_00292_amd", (".py", ".cpp", ".h", ".hip")):
        s = open(p).read()
        assert not re.search(r"^\s*(import|from)\s+oracle\b", s, re.M), p
        assert "rt_oracle" not in s, p
    for p in _sources("oracle", (".py", ".c", ".h")):
        s = open(p).read()
        assert "paper_2603_00292_amd" not in s, p
        assert "rt_layout" not in s and "rt_kernels" not in s, p


def test_autotune_cache_roundtrip(tmp_path, monkeypatch):
    """The autotuner's JSON cache (host logic): keyed by device and scene
    class (powers of four of the triangle and ray counts), atomic rewrite,
    choices of other classes and devices kept."""
    from paper_2603_00292_amd import autotune

    monkeypatch.setenv("RTQ_AUTOTUNE_CACHE", str(tmp_path / "sub" / "tune.json"))
    assert autotune.scene_class(1_310_720, 4_194_304) == "tri4^10_ray4^11"
    assert autotune.scene_class(4096, 65536) == "tri4^6_ray4^8"
    assert autotune.cached_choice("gfx950_cu256", "tri4^10_ray4^11") is None
    a = {"node_width": 4, "stack_entries": 16, "workgroup": 256, "ms": 1.9}
    b = {"node_width": 8, "stack_entries": 32, "workgroup": 128, "ms": 0.1}
    autotune.save_choice("gfx950_cu256", "tri4^10_ray4^11", a)
    autotune.save_choice("gfx950_cu256", "tri4^6_ray4^8", b)
    autotune.save_choice("gfx942_cu304", "tri4^10_ray4^11", b)
    assert autotune.cached_choice("gfx950_cu256", "tri4^10_ray4^11") == a
    assert autotune.cached_choice("gfx950_cu256", "tri4^6_ray4^8") == b
    assert autotune.cached_choice("gfx942_cu304", "tri4^10_ray4^11") == b
    assert not [p for p in (tmp_path / "sub").iterdir() if ".tmp" in p.name]


@pytest.mark.parametrize("content", ["", "{not json", "[1, 2]", '{"gfx950_cu256": 3}', "\x00\x01",
                                     '{"gfx950_cu256": {"tri4^10_ray4^11": 5}}',
                                     '{"gfx950_cu256": {"tri4^10_ray4^11": {"node_width": 4}}}'])
def test_autotune_cache_malformed_reads_empty(tmp_path, monkeypatch, content):
    """A truncated or malformed cache file reads as empty, and the next save
    replaces it with a valid one."""
    from paper_2603_00292_amd import autotune

    p = tmp_path / "tune.json"
    p.write_text(content)
    monkeypatch.setenv("RTQ_AUTOTUNE_CACHE", str(p))
    assert autotune.cached_choice("gfx950_cu256", "tri4^10_ray4^11") is None
    a = {"node_width": 4, "stack_entries": 16, "workgroup": 256, "ms": 1.9}
    autotune.save_choice("gfx950_cu256", "tri4^10_ray4^11", a)
    assert autotune.cached_choice("gfx950_cu256", "tri4^10_ray4^11") == a
