"""CPU checks of the C ABI library: it loads, exports every symbol that
include/cyrus.h declares, and validates configurations before touching a
device (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_2506_00167_amd import cyrus
from paper_2506_00167_amd import workload as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(cyrus.LIB_PATH):
        from paper_2506_00167_amd import build
        build.build()
    return cyrus.lib()


def _header_functions():
    text = open(os.path.join(ROOT, "include", "cyrus.h")).read()
    return sorted(set(re.findall(r"\b(cyrus_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    declared = _header_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in cyrus.h but not exported"
    assert set(declared) == set(cyrus.SYMBOLS)


def test_workspace_sizes(lib):
    for cfg in (wl.TINY, wl.TREE_E8K3, wl.STRESS_E16K4, wl.PAPER_DEPTH1):
        d, h = cyrus.cyrus_codebook_workspace_size(cyrus.make_config(cfg))
        assert d >= 2 * cfg.num_nodes * cfg.num_ue and h >= cfg.num_nodes * cfg.num_ue
        d2, h2 = cyrus.cyrus_codebook_workspace_size(cyrus.make_config(cfg, export_logits=True))
        assert d2 >= d + 4 * cfg.num_nodes * cfg.num_ue and h2 >= h + 4 * cfg.num_nodes * cfg.num_ue


@pytest.mark.parametrize("field,value,status", [
    ("num_ue", 0, -2), ("num_ue", 33, -2), ("max_arrival", 8, -2), ("num_minislots", 0, -2),
    ("rb_per_unit", 0, -2), ("num_hidden", 5, -2), ("precision", 7, -1), ("flags", 64, -1),
])
def test_config_validation(lib, field, value, status):
    c = cyrus.make_config(wl.TREE_E8K3)
    setattr(c, field, value)
    with pytest.raises(cyrus.CyrusError) as ei:
        cyrus.cyrus_codebook_workspace_size(c)
    assert ei.value.status == status
    assert cyrus.cyrus_last_error()


def test_hidden_width_and_state_range(lib):
    c = cyrus.make_config(wl.TREE_E8K3)
    c.hidden[0] = 200
    with pytest.raises(cyrus.CyrusError):
        cyrus.cyrus_codebook_workspace_size(c)
    c = cyrus.make_config(wl.TreeConfig(num_ue=4, max_arrival=7, num_minislots=7, rb_per_unit=6))
    with pytest.raises(cyrus.CyrusError):  # 7*7*6 > 255
        cyrus.cyrus_codebook_workspace_size(c)


def test_null_handles_are_safe(lib):
    assert lib.cyrus_codebook_num_nodes(None) == -1
    assert lib.cyrus_codebook_kernel_path(None) == b"none"
    lib.cyrus_codebook_destroy(None)
    assert lib.cyrus_codebook_wait(None) == -1
    assert lib.cyrus_status_string(-3) == b"workspace too small or misplaced"


def test_create_rejects_host_memory_as_workspace(lib):
    # the pointer checks run before anything is enqueued
    cfg = cyrus.make_config(wl.TINY)
    d, h = cyrus.cyrus_codebook_workspace_size(cfg)
    buf = ctypes.create_string_buffer(d + 256)
    addr = (ctypes.addressof(buf) + 255) // 256 * 256
    w = cyrus._WeightsView(wl.make_weights(wl.TINY, 1))
    out = ctypes.c_void_p()
    rc = lib.cyrus_codebook_create(ctypes.byref(cfg), ctypes.byref(w.struct), addr, d, addr, h, None,
                                   ctypes.byref(out))
    assert rc in (-3, -4)
    assert out.value is None
