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
    for bad in (200, 16, 544, 0):
        c = cyrus.make_config(wl.TREE_E8K3)
        c.hidden[0] = bad
        with pytest.raises(cyrus.CyrusError) as ei:
            cyrus.cyrus_codebook_workspace_size(c)
        assert ei.value.status == -2
    # multiples of 32 are accepted: they are computed zero-padded to 128
    sizes = {}
    for width in (32, 96, 128, 160, 256, 480, 512):
        c = cyrus.make_config(wl.TREE_E8K3)
        c.hidden[0] = c.hidden[1] = width
        sizes[width] = cyrus.cyrus_codebook_workspace_size(c)[0]
    assert sizes[32] == sizes[96] == sizes[128] < sizes[160] == sizes[256] < sizes[480] == sizes[512]
    c = cyrus.make_config(wl.TreeConfig(num_ue=4, max_arrival=7, num_minislots=7, rb_per_unit=6))
    with pytest.raises(cyrus.CyrusError):  # 7*7*6 > 255
        cyrus.cyrus_codebook_workspace_size(c)


def test_critic_hidden_widths(lib):
    # multiples of 32 in [32, 512] are accepted (zero-padded to the next
    # multiple of 128 inside); anything else is refused before a device is used
    def size(actor, critic):
        c = cyrus.make_critic_config(wl.CriticConfig(num_ue=4, max_arrival=2, num_minislots=7, num_samples=16,
                                                     actor_hidden=actor, critic_hidden=critic))
        d = ctypes.c_size_t()
        rc = lib.cyrus_critic_workspace_size(ctypes.byref(c), ctypes.byref(d))
        return rc, d.value
    ok = {w: size((w, w), (w, w)) for w in (32, 96, 128, 160, 256, 480, 512)}
    assert all(rc == 0 for rc, _ in ok.values())
    assert ok[32][1] == ok[96][1] == ok[128][1] < ok[160][1] == ok[256][1] < ok[480][1] == ok[512][1]
    for bad in (0, 16, 100, 544, 1024):
        assert size((bad,), (128,))[0] == -2
        assert size((128,), (128, bad))[0] == -2


def test_null_handles_are_safe(lib):
    assert lib.cyrus_codebook_num_nodes(None) == -1
    assert lib.cyrus_codebook_kernel_path(None) == b"none"
    lib.cyrus_codebook_destroy(None)
    assert lib.cyrus_codebook_wait(None) == -1
    assert lib.cyrus_status_string(-3) == b"workspace too small or misplaced"
    assert lib.cyrus_engine_run(None, 0, None, None, None, None, None) == -1
    assert lib.cyrus_engine_set_level_lag(None, 0) == -1


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


def test_library_matches_its_sources(lib):
    from paper_2506_00167_amd import build
    lib.cyrus_build_source_hash.restype = ctypes.c_char_p
    assert lib.cyrus_build_source_hash().decode() == build.source_hash()


def test_stale_library_is_refused(monkeypatch):
    """A library built from other sources than those beside it is refused,
    so a stale binary cannot be tested or benchmarked silently."""
    from paper_2506_00167_amd import build
    if not os.path.exists(cyrus.LIB_PATH):
        build.build()
    monkeypatch.setattr(build, "source_hash", lambda: "0000000000000000")
    monkeypatch.setattr(cyrus, "_lib", None)
    with pytest.raises(RuntimeError, match="other sources"):
        cyrus.lib()


def test_batch_argument_checks(lib):
    """Both batch entry points validate before enqueueing anything."""
    vp = ctypes.c_void_p
    hs = (vp * 1)(None)
    ues = (cyrus.cyrus_ue_state * 1)()
    assert lib.cyrus_codebook_build_batch(hs, ues, 0, None) == -2
    assert lib.cyrus_codebook_build_batch(hs, ues, 129, None) == -2
    assert lib.cyrus_codebook_build_batch(hs, ues, 1, None) == -1   # NULL handle
    assert lib.cyrus_codebook_build_batch(None, ues, 1, None) == -1
    assert lib.cyrus_codebook_build_batch_device(hs, (vp * 1)(None), 0, None) == -2
    assert lib.cyrus_codebook_build_batch_device(hs, (vp * 1)(None), 1, None) == -1
