"""Python binding of libcyrus (the C ABI in include/cyrus.h).

Argument marshalling only: every step of the codebook build runs in the HIP
library. PyTorch provides the device workspace, the pinned host buffer and the
stream handle. The functions named like the C entry points are one-to-one
wrappers; ``Codebook`` owns the buffers of one builder.

The library must be built first (``python -m paper_2506_00167_amd.build``);
loading fails loudly if it is missing, there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from .workload import TreeConfig, UEState

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcyrus.so")

CYRUS_OK = 0
STATUS = {0: "OK", -1: "EINVAL", -2: "ERANGE", -3: "EWORKSPACE", -4: "EDEVICE", -5: "ENOTREADY", -6: "EUNSUPPORTED"}
PRECISION = {"fp32": 0, "bf16": 1, "fp8": 2}
FLAG_EXPORT_LOGITS = 1
FLAG_LEVEL_KERNEL = 2
FLAG_HUNTINGTON_HILL = 4
FLAG_GAUSSIAN_HEAD = 8
MAX_HIDDEN = 4
MAX_LAYERS = 5

SYMBOLS = (
    "cyrus_codebook_workspace_size", "cyrus_codebook_create", "cyrus_codebook_set_weights",
    "cyrus_codebook_build", "cyrus_codebook_build_device", "cyrus_codebook_build_batch",
    "cyrus_codebook_build_batch_device", "cyrus_build_source_hash",
    "cyrus_codebook_wait", "cyrus_codebook_lookup", "cyrus_codebook_assemble", "cyrus_codebook_export", "cyrus_codebook_device_alloc",
    "cyrus_codebook_num_nodes", "cyrus_codebook_kernel_path", "cyrus_codebook_set_rng", "cyrus_codebook_destroy",
    "cyrus_status_string", "cyrus_last_error",
    "cyrus_critic_workspace_size", "cyrus_critic_create", "cyrus_critic_evaluate", "cyrus_critic_evaluate_noalloc",
    "cyrus_critic_destroy",
    "cyrus_engine_create", "cyrus_engine_submit", "cyrus_engine_step", "cyrus_engine_set_levels_per_step",
    "cyrus_engine_set_resident", "cyrus_engine_set_level_lag",
    "cyrus_engine_poll",
    "cyrus_engine_completed", "cyrus_engine_result", "cyrus_engine_run", "cyrus_engine_stats",
    "cyrus_engine_destroy",
)
REQ_WAITING, REQ_RUNNING, REQ_DONE = 0, 1, 2


class CyrusError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} ({status}): {msg}")
        self.status = status


class cyrus_config(ctypes.Structure):
    _fields_ = [("num_ue", ctypes.c_int32), ("max_arrival", ctypes.c_int32), ("num_minislots", ctypes.c_int32),
                ("rb_per_unit", ctypes.c_int32), ("num_hidden", ctypes.c_int32),
                ("hidden", ctypes.c_int32 * MAX_HIDDEN), ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


_f32p = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class cyrus_weights(ctypes.Structure):
    _fields_ = [("w", _f32p * MAX_LAYERS), ("b", _f32p * MAX_LAYERS), ("act_scale", _f32p)]


class cyrus_critic_config(ctypes.Structure):
    _fields_ = [("num_ue", ctypes.c_int32), ("num_minislots", ctypes.c_int32), ("num_samples", ctypes.c_int32),
                ("actor_hidden_layers", ctypes.c_int32), ("actor_hidden", ctypes.c_int32 * MAX_HIDDEN),
                ("critic_hidden_layers", ctypes.c_int32), ("critic_hidden", ctypes.c_int32 * MAX_HIDDEN),
                ("discount", ctypes.c_float), ("entropy_coef", ctypes.c_float)]


class cyrus_critic_weights(ctypes.Structure):
    _fields_ = [("actor", cyrus_weights), ("q", cyrus_weights * 2), ("q_targ", cyrus_weights * 2)]


class cyrus_critic_batch(ctypes.Structure):
    _fields_ = [("ue", _i32p), ("k", _i32p), ("c", _u8p), ("y", _f32p), ("reward", _f32p)]


class cyrus_ue_state(ctypes.Structure):
    _fields_ = [("rb", _i32p), ("mcs", _i32p), ("sinr_db", _f32p)]


_lib = None


def lib():
    """Load libcyrus.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_00167_amd.build`")
        # torch brings its own HIP runtime; loading it first makes libcyrus
        # bind to that same runtime (one runtime per process, so pointers
        # allocated by torch are known to the library)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.cyrus_build_source_hash.restype = ctypes.c_char_p
        built = L.cyrus_build_source_hash().decode()
        from . import build as _build
        want = _build.source_hash()
        if built != want:
            raise RuntimeError(f"{LIB_PATH} was built from other sources (hash {built}, sources {want}): "
                               "rebuild it with `python -m paper_2506_00167_amd.build`")
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.cyrus_codebook_workspace_size.argtypes = [ctypes.POINTER(cyrus_config), ctypes.POINTER(sz),
                                                    ctypes.POINTER(sz)]
        L.cyrus_codebook_create.argtypes = [ctypes.POINTER(cyrus_config), ctypes.POINTER(cyrus_weights), vp, sz, vp,
                                            sz, vp, ctypes.POINTER(vp)]
        L.cyrus_codebook_set_weights.argtypes = [vp, ctypes.POINTER(cyrus_weights), vp]
        L.cyrus_codebook_build.argtypes = [vp, ctypes.POINTER(cyrus_ue_state), vp]
        L.cyrus_codebook_build_device.argtypes = [vp, vp, vp]
        L.cyrus_codebook_build_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(cyrus_ue_state), ctypes.c_int32,
                                                 vp]
        L.cyrus_codebook_build_batch_device.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int32, vp]
        L.cyrus_codebook_wait.argtypes = [vp]
        L.cyrus_codebook_lookup.argtypes = [vp, _u8p, ctypes.c_int32, _u8p]
        L.cyrus_codebook_export.argtypes = [vp, _u8p, _f32p]
        L.cyrus_codebook_assemble.argtypes = [vp, _i32p, ctypes.c_int32, _u8p, _u8p, ctypes.POINTER(ctypes.c_int32)]
        L.cyrus_codebook_device_alloc.argtypes = [vp]
        L.cyrus_codebook_device_alloc.restype = vp
        L.cyrus_codebook_num_nodes.argtypes = [vp]
        L.cyrus_codebook_num_nodes.restype = ctypes.c_int64
        L.cyrus_codebook_kernel_path.argtypes = [vp]
        L.cyrus_codebook_kernel_path.restype = ctypes.c_char_p
        L.cyrus_codebook_set_rng.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint64]
        L.cyrus_critic_workspace_size.argtypes = [ctypes.POINTER(cyrus_critic_config), ctypes.POINTER(sz)]
        L.cyrus_critic_create.argtypes = [ctypes.POINTER(cyrus_critic_config), ctypes.POINTER(cyrus_critic_weights),
                                          vp, sz, vp, ctypes.POINTER(vp)]
        L.cyrus_critic_evaluate.argtypes = [vp, ctypes.POINTER(cyrus_critic_batch), ctypes.c_uint64, ctypes.c_uint64,
                                            vp, vp, vp, vp]
        L.cyrus_critic_evaluate_noalloc.argtypes = [vp, ctypes.POINTER(cyrus_critic_batch), ctypes.c_uint64,
                                                    ctypes.c_uint64, vp, vp, vp, vp]
        L.cyrus_engine_set_resident.argtypes = [vp, ctypes.c_int32]
        L.cyrus_critic_destroy.argtypes = [vp]
        L.cyrus_critic_destroy.restype = None
        L.cyrus_codebook_destroy.argtypes = [vp]
        L.cyrus_codebook_destroy.restype = None
        L.cyrus_status_string.argtypes = [ctypes.c_int]
        L.cyrus_status_string.restype = ctypes.c_char_p
        L.cyrus_last_error.argtypes = []
        L.cyrus_last_error.restype = ctypes.c_char_p
        L.cyrus_engine_create.argtypes = [vp, sz, vp, sz, ctypes.c_int32, vp, ctypes.POINTER(vp)]
        L.cyrus_engine_submit.argtypes = [vp, vp, ctypes.POINTER(cyrus_ue_state), ctypes.POINTER(ctypes.c_int64)]
        L.cyrus_engine_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.cyrus_engine_set_levels_per_step.argtypes = [vp, ctypes.c_int32]
        L.cyrus_engine_set_level_lag.argtypes = [vp, ctypes.c_int32]
        L.cyrus_engine_poll.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_double)]
        L.cyrus_engine_completed.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                             ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.cyrus_engine_result.argtypes = [vp, ctypes.c_int64, _u8p, sz]
        L.cyrus_engine_run.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(cyrus_ue_state),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(vp),
                                       ctypes.POINTER(ctypes.c_double)]
        L.cyrus_engine_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
        L.cyrus_engine_destroy.argtypes = [vp]
        L.cyrus_engine_destroy.restype = None
        for name in SYMBOLS:
            if name not in ("cyrus_codebook_device_alloc", "cyrus_codebook_num_nodes", "cyrus_codebook_kernel_path",
                            "cyrus_codebook_destroy", "cyrus_status_string", "cyrus_last_error",
                            "cyrus_engine_destroy"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != CYRUS_OK:
        raise CyrusError(rc, where, lib().cyrus_last_error().decode())


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def make_config(cfg: TreeConfig, export_logits: bool = False, force_level: bool = False) -> cyrus_config:
    c = cyrus_config()
    c.num_ue = cfg.num_ue
    c.max_arrival = cfg.max_arrival
    c.num_minislots = cfg.num_minislots
    c.rb_per_unit = cfg.rb_per_unit
    c.num_hidden = len(cfg.hidden)
    for i, h in enumerate(cfg.hidden):
        c.hidden[i] = h
    c.precision = PRECISION[cfg.precision]
    if cfg.rounding not in ("lr", "hh"):
        raise ValueError(f"rounding must be 'lr' or 'hh', not {cfg.rounding!r}")
    if cfg.head not in ("softmax", "gaussian"):
        raise ValueError(f"head must be 'softmax' or 'gaussian', not {cfg.head!r}")
    c.flags = ((FLAG_EXPORT_LOGITS if export_logits else 0) | (FLAG_LEVEL_KERNEL if force_level else 0)
               | (FLAG_HUNTINGTON_HILL if cfg.rounding == "hh" else 0)
               | (FLAG_GAUSSIAN_HEAD if cfg.head == "gaussian" else 0))
    return c


class _WeightsView:
    """Keeps the float32 arrays referenced while the C struct points at them."""

    def __init__(self, weights, act_scale=None):
        self.arrays = []
        self.struct = cyrus_weights()
        for l, (w, b) in enumerate(weights):
            w = np.ascontiguousarray(w, dtype=np.float32)
            b = np.ascontiguousarray(b, dtype=np.float32)
            self.arrays += [w, b]
            self.struct.w[l] = w.ctypes.data_as(_f32p)
            self.struct.b[l] = b.ctypes.data_as(_f32p)
        if act_scale is not None:
            a = np.ascontiguousarray(act_scale, dtype=np.float32)
            self.arrays.append(a)
            self.struct.act_scale = a.ctypes.data_as(_f32p)


# ------------------------------------------------------- same-name wrappers

def cyrus_codebook_workspace_size(cfg: cyrus_config):
    d, h = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().cyrus_codebook_workspace_size(ctypes.byref(cfg), ctypes.byref(d), ctypes.byref(h)),
           "cyrus_codebook_workspace_size")
    return d.value, h.value


def cyrus_codebook_create(cfg: cyrus_config, w: cyrus_weights, ws_ptr: int, ws_bytes: int, host_ptr: int,
                          host_bytes: int, stream) -> int:
    out = ctypes.c_void_p()
    _check(lib().cyrus_codebook_create(ctypes.byref(cfg), ctypes.byref(w), ws_ptr, ws_bytes, host_ptr, host_bytes,
                                       _stream_ptr(stream), ctypes.byref(out)), "cyrus_codebook_create")
    return out.value


def cyrus_codebook_set_weights(h: int, w: cyrus_weights, stream) -> None:
    _check(lib().cyrus_codebook_set_weights(h, ctypes.byref(w), _stream_ptr(stream)), "cyrus_codebook_set_weights")


def cyrus_codebook_build(h: int, ue: cyrus_ue_state, stream) -> None:
    _check(lib().cyrus_codebook_build(h, ctypes.byref(ue), _stream_ptr(stream)), "cyrus_codebook_build")


def cyrus_codebook_build_device(h: int, ue_dev_ptr: int, stream) -> None:
    _check(lib().cyrus_codebook_build_device(h, ue_dev_ptr, _stream_ptr(stream)), "cyrus_codebook_build_device")


def cyrus_codebook_build_batch(handles: Sequence[int], ues: Sequence[cyrus_ue_state], stream) -> None:
    n = len(handles)
    hs = (ctypes.c_void_p * n)(*handles)
    us = (cyrus_ue_state * n)(*ues)
    _check(lib().cyrus_codebook_build_batch(hs, us, n, _stream_ptr(stream)), "cyrus_codebook_build_batch")


def cyrus_codebook_build_batch_device(handles: Sequence[int], ue_dev_ptrs: Sequence[int], stream) -> None:
    n = len(handles)
    hs = (ctypes.c_void_p * n)(*handles)
    us = (ctypes.c_void_p * n)(*ue_dev_ptrs)
    _check(lib().cyrus_codebook_build_batch_device(hs, us, n, _stream_ptr(stream)),
           "cyrus_codebook_build_batch_device")


def cyrus_codebook_wait(h: int) -> None:
    _check(lib().cyrus_codebook_wait(h), "cyrus_codebook_wait")


def cyrus_codebook_lookup(h: int, arrivals: Sequence[int], num_ue: int) -> np.ndarray:
    arr = np.ascontiguousarray(arrivals, dtype=np.uint8)
    out = np.zeros(num_ue, dtype=np.uint8)
    _check(lib().cyrus_codebook_lookup(h, arr.ctypes.data_as(_u8p), arr.size, out.ctypes.data_as(_u8p)),
           "cyrus_codebook_lookup")
    return out


def cyrus_codebook_assemble(h: int, raw, carry_in: int, num_minislots: int, num_ue: int):
    raw = np.ascontiguousarray(raw, dtype=np.int32)
    served = np.zeros(num_minislots, dtype=np.uint8)
    y = np.zeros((num_minislots, num_ue), dtype=np.uint8)
    co = ctypes.c_int32()
    _check(lib().cyrus_codebook_assemble(h, raw.ctypes.data_as(_i32p), int(carry_in), served.ctypes.data_as(_u8p),
                                         y.ctypes.data_as(_u8p), ctypes.byref(co)), "cyrus_codebook_assemble")
    return served, y, co.value


def cyrus_codebook_export(h: int, nodes: int, num_ue: int, logits: bool):
    alloc = np.zeros((nodes, num_ue), dtype=np.uint8)
    lg = np.zeros((nodes, num_ue), dtype=np.float32) if logits else None
    _check(lib().cyrus_codebook_export(h, alloc.ctypes.data_as(_u8p), None if lg is None else lg.ctypes.data_as(_f32p)),
           "cyrus_codebook_export")
    return alloc, lg


def cyrus_codebook_device_alloc(h: int) -> int:
    return lib().cyrus_codebook_device_alloc(h)


def cyrus_codebook_num_nodes(h: int) -> int:
    return lib().cyrus_codebook_num_nodes(h)


def cyrus_codebook_kernel_path(h: int) -> str:
    return lib().cyrus_codebook_kernel_path(h).decode()


def cyrus_codebook_destroy(h: int) -> None:
    lib().cyrus_codebook_destroy(h)


def cyrus_status_string(status: int) -> str:
    return lib().cyrus_status_string(status).decode()


def cyrus_last_error() -> str:
    return lib().cyrus_last_error().decode()


# ------------------------------------------------------------- convenience

def ue_struct(ue: UEState):
    rb = np.ascontiguousarray(ue.rb, dtype=np.int32)
    mcs = np.ascontiguousarray(ue.mcs, dtype=np.int32)
    sinr = np.ascontiguousarray(ue.sinr_db, dtype=np.float32)
    s = cyrus_ue_state(rb.ctypes.data_as(_i32p), mcs.ctypes.data_as(_i32p), sinr.ctypes.data_as(_f32p))
    return s, (rb, mcs, sinr)


def ue_device_tensor(ue: UEState, device="cuda"):
    """Device copy of a UE state in the layout of cyrus_codebook_build_device:
    int32 rb[E], int32 mcs[E], float32 sinr_db[E] (as raw bits)."""
    import torch
    packed = np.concatenate([np.asarray(ue.rb, np.int32), np.asarray(ue.mcs, np.int32),
                             np.asarray(ue.sinr_db, np.float32).view(np.int32)])
    return torch.from_numpy(packed).to(device)


class Codebook:
    """One codebook builder with its caller-owned buffers (torch device memory
    for the workspace, pinned host memory for the mirror)."""

    def __init__(self, cfg: TreeConfig, weights, act_scale=None, export_logits: bool = False,
                 force_level: bool = False, device: str = "cuda", stream=None):
        import torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.cconf = make_config(cfg, export_logits, force_level)
        self.export_logits = export_logits
        self.ws_bytes, self.host_bytes = cyrus_codebook_workspace_size(self.cconf)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.host = torch.empty(self.host_bytes, dtype=torch.uint8, pin_memory=True)
        self._w = _WeightsView(weights, act_scale)
        self.weights, self.act_scale = weights, act_scale
        self.stream = stream
        with torch.cuda.device(self.device):
            self.handle = cyrus_codebook_create(self.cconf, self._w.struct, self.ws.data_ptr(), self.ws_bytes,
                                                self.host.data_ptr(), self.host_bytes, stream)
        self.num_nodes = cyrus_codebook_num_nodes(self.handle)
        self._ue_keep = None

    @property
    def kernel_path(self) -> str:
        return cyrus_codebook_kernel_path(self.handle)

    def set_rng(self, seed: int, tti: int):
        """Gaussian head: Philox key and TTI number of the following builds."""
        _check(lib().cyrus_codebook_set_rng(self.handle, int(seed) & 0xFFFFFFFFFFFFFFFF,
                                            int(tti) & 0xFFFFFFFFFFFFFFFF), "cyrus_codebook_set_rng")
        return self

    def set_weights(self, weights, act_scale=None):
        view = _WeightsView(weights, act_scale)
        cyrus_codebook_set_weights(self.handle, view.struct, self.stream)
        # only a refresh that took effect replaces the weights this handle reports
        self._w = view
        self.weights, self.act_scale = weights, act_scale

    def build(self, ue: UEState):
        s, keep = ue_struct(ue)
        cyrus_codebook_build(self.handle, s, self.stream)
        return self

    def build_device(self, ue_dev):
        self._ue_keep = ue_dev
        cyrus_codebook_build_device(self.handle, ue_dev.data_ptr(), self.stream)
        return self

    def wait(self):
        cyrus_codebook_wait(self.handle)

    def lookup(self, arrivals) -> np.ndarray:
        return cyrus_codebook_lookup(self.handle, arrivals, self.cfg.num_ue)

    def assemble(self, raw_arrivals, carry_in: int = 0):
        """Controller + Alg. 3: (served [M], Y [M,E], carry_out)."""
        return cyrus_codebook_assemble(self.handle, raw_arrivals, carry_in, self.cfg.num_minislots, self.cfg.num_ue)

    def export(self):
        return cyrus_codebook_export(self.handle, self.num_nodes, self.cfg.num_ue, self.export_logits)

    def device_alloc_ptr(self) -> int:
        return cyrus_codebook_device_alloc(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            cyrus_codebook_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_batch(codebooks: Sequence[Codebook], ues: Sequence[UEState], stream=None):
    """Host UE states in, every codebook in its pinned mirror after the wait."""
    structs = [ue_struct(u) for u in ues]  # the arrays stay referenced for the call
    cyrus_codebook_build_batch([c.handle for c in codebooks], [st for st, _ in structs], stream)


def build_batch_device(codebooks: Sequence[Codebook], ue_devs, stream=None):
    """Device UE states (ue_device_tensor) in, codebooks left on the device."""
    cyrus_codebook_build_batch_device([c.handle for c in codebooks], [u.data_ptr() for u in ue_devs], stream)


# ------------------------------------------------------------ serving engine

def cyrus_engine_create(dev_ptr: int, dev_bytes: int, host_ptr: int, host_bytes: int, max_active: int,
                        stream) -> int:
    out = ctypes.c_void_p()
    _check(lib().cyrus_engine_create(dev_ptr, dev_bytes, host_ptr, host_bytes, max_active, _stream_ptr(stream),
                                     ctypes.byref(out)), "cyrus_engine_create")
    return out.value


def cyrus_engine_submit(eng: int, cell: int, ue: cyrus_ue_state) -> int:
    t = ctypes.c_int64()
    _check(lib().cyrus_engine_submit(eng, cell, ctypes.byref(ue), ctypes.byref(t)), "cyrus_engine_submit")
    return t.value


def cyrus_engine_step(eng: int):
    r, w = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().cyrus_engine_step(eng, ctypes.byref(r), ctypes.byref(w)), "cyrus_engine_step")
    return r.value, w.value


def cyrus_engine_poll(eng: int, ticket: int):
    st, lat = ctypes.c_int32(), ctypes.c_double()
    _check(lib().cyrus_engine_poll(eng, ticket, ctypes.byref(st), ctypes.byref(lat)), "cyrus_engine_poll")
    return st.value, lat.value


def cyrus_engine_completed(eng: int, cap: int = 256):
    t = (ctypes.c_int64 * cap)()
    lat = (ctypes.c_double * cap)()
    n = ctypes.c_int32()
    _check(lib().cyrus_engine_completed(eng, t, lat, cap, ctypes.byref(n)), "cyrus_engine_completed")
    return [(t[i], lat[i]) for i in range(n.value)]


def cyrus_engine_result(eng: int, ticket: int, nodes: int, num_ue: int) -> np.ndarray:
    out = np.zeros((nodes, num_ue), dtype=np.uint8)
    _check(lib().cyrus_engine_result(eng, ticket, out.ctypes.data_as(_u8p), out.nbytes), "cyrus_engine_result")
    return out


def cyrus_engine_run(eng: int, cells: Sequence[int], ues: Sequence[cyrus_ue_state], arrival_us,
                     results: Optional[Sequence[int]] = None) -> np.ndarray:
    """Native request loop; returns the latency of each request in us."""
    n = len(cells)
    hs = (ctypes.c_void_p * n)(*cells)
    us = (cyrus_ue_state * n)(*ues)
    arr = np.ascontiguousarray(arrival_us, dtype=np.float64)
    lat = np.zeros(n, dtype=np.float64)
    res = (ctypes.c_void_p * n)(*results) if results is not None else None
    _check(lib().cyrus_engine_run(eng, n, hs, us, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), res,
                                  lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "cyrus_engine_run")
    return lat


def cyrus_engine_stats(eng: int) -> dict:
    c = (ctypes.c_int64 * 7)()
    _check(lib().cyrus_engine_stats(eng, c, 7), "cyrus_engine_stats")
    keys = ("submitted", "completed", "steps", "deferred_memory", "deferred_batch", "pool_bytes_used",
            "pool_bytes_peak")
    return dict(zip(keys, list(c)))


def cyrus_engine_destroy(eng: int) -> None:
    lib().cyrus_engine_destroy(eng)


class Engine:
    """Continuous-batching engine over caller-owned pools (torch device memory
    and pinned host memory). Cells are Codebook objects (their weights)."""

    def __init__(self, device_pool_bytes: int, host_pool_bytes: int, max_active: int = 64, device: str = "cuda",
                 stream=None, resident: bool = False):
        import torch
        self.dpool = torch.empty(device_pool_bytes, dtype=torch.uint8, device=device)
        self.hpool = torch.empty(host_pool_bytes, dtype=torch.uint8, pin_memory=True)
        self.stream = stream
        self.handle = cyrus_engine_create(self.dpool.data_ptr(), device_pool_bytes, self.hpool.data_ptr(),
                                          host_pool_bytes, max_active, stream)
        self._cells = {}
        self.resident = bool(resident)
        if resident:
            _check(lib().cyrus_engine_set_resident(self.handle, 1), "cyrus_engine_set_resident")

    def submit(self, cell: Codebook, ue: UEState) -> int:
        s, keep = ue_struct(ue)
        t = cyrus_engine_submit(self.handle, cell.handle, s)
        self._cells[t] = cell
        return t

    def step(self):
        return cyrus_engine_step(self.handle)

    def set_level_lag(self, lag: int):
        _check(lib().cyrus_engine_set_level_lag(self.handle, int(lag)), "cyrus_engine_set_level_lag")
        return self

    def set_levels_per_step(self, levels: int):
        _check(lib().cyrus_engine_set_levels_per_step(self.handle, int(levels)), "cyrus_engine_set_levels_per_step")
        return self

    def poll(self, ticket: int):
        return cyrus_engine_poll(self.handle, ticket)

    def completed(self):
        """[(ticket, latency_us)] of requests finished since the last call."""
        return cyrus_engine_completed(self.handle)

    def result(self, ticket: int) -> np.ndarray:
        cell = self._cells.pop(ticket)
        return cyrus_engine_result(self.handle, ticket, cell.num_nodes, cell.cfg.num_ue)

    def run(self, cells: Sequence[Codebook], ues: Sequence[UEState], arrival_us, keep_results: bool = False):
        """cyrus_engine_run: the whole request stream in the library's own
        loop. Returns (latency_us per request, codebooks or None)."""
        structs = [ue_struct(u) for u in ues]  # the arrays stay referenced for the call
        outs = [np.zeros((c.num_nodes, c.cfg.num_ue), dtype=np.uint8) for c in cells] if keep_results else None
        lat = cyrus_engine_run(self.handle, [c.handle for c in cells], [st for st, _ in structs], arrival_us,
                               [o.ctypes.data for o in outs] if keep_results else None)
        return lat, outs

    def stats(self) -> dict:
        return cyrus_engine_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            cyrus_engine_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



# ------------------------------------------------------------------- critic

def make_critic_config(cfg) -> cyrus_critic_config:
    c = cyrus_critic_config()
    c.num_ue = cfg.num_ue
    c.num_minislots = cfg.num_minislots
    c.num_samples = cfg.num_samples
    c.actor_hidden_layers = len(cfg.actor_hidden)
    for i, h in enumerate(cfg.actor_hidden):
        c.actor_hidden[i] = h
    c.critic_hidden_layers = len(cfg.critic_hidden)
    for i, h in enumerate(cfg.critic_hidden):
        c.critic_hidden[i] = h
    c.discount = cfg.discount
    c.entropy_coef = cfg.entropy_coef
    return c


class Critic:
    """The Near-RT RIC critic pass (cyrus_critic_*): one actor with the Gaussian
    head and four critics, FP32, in a caller-owned torch device workspace."""

    def __init__(self, cfg, actor_w, q_w, qt_w, device: str = "cuda", stream=None):
        import torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.cconf = make_critic_config(cfg)
        d = ctypes.c_size_t()
        _check(lib().cyrus_critic_workspace_size(ctypes.byref(self.cconf), ctypes.byref(d)),
               "cyrus_critic_workspace_size")
        self.ws = torch.empty(d.value, dtype=torch.uint8, device=self.device)
        self._views = [_WeightsView(actor_w)] + [_WeightsView(w) for w in q_w] + [_WeightsView(w) for w in qt_w]
        cw = cyrus_critic_weights()
        cw.actor = self._views[0].struct
        cw.q[0], cw.q[1] = self._views[1].struct, self._views[2].struct
        cw.q_targ[0], cw.q_targ[1] = self._views[3].struct, self._views[4].struct
        self._cw = cw
        self.stream = stream
        out = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().cyrus_critic_create(ctypes.byref(self.cconf), ctypes.byref(cw), self.ws.data_ptr(), d.value,
                                             _stream_ptr(stream), ctypes.byref(out)), "cyrus_critic_create")
        self.handle = out.value
        H, M = cfg.num_samples, cfg.num_minislots
        self.q = torch.empty((2, H, M), dtype=torch.float32, device=self.device)
        self.qhat = torch.empty((H, M), dtype=torch.float32, device=self.device)
        self.loss = torch.empty(2, dtype=torch.float32, device=self.device)

    def evaluate(self, batch, seed: int, episode: int):
        """batch: device tensors (ue [H,3E] i32, k [H,M] i32, c [H,M,E] u8, y [H,M,E]
        f32, r [H] f32). Returns the output tensors (q [2,H,M], qhat [H,M], loss [2]),
        written asynchronously on the handle's stream."""
        ue, k, c, y, r = batch
        self._keep = batch
        b = cyrus_critic_batch(ctypes.cast(ue.data_ptr(), _i32p), ctypes.cast(k.data_ptr(), _i32p),
                               ctypes.cast(c.data_ptr(), _u8p), ctypes.cast(y.data_ptr(), _f32p),
                               ctypes.cast(r.data_ptr(), _f32p))
        _check(lib().cyrus_critic_evaluate(self.handle, ctypes.byref(b), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                           int(episode) & 0xFFFFFFFFFFFFFFFF, self.q.data_ptr(), self.qhat.data_ptr(),
                                           self.loss.data_ptr(), _stream_ptr(self.stream)), "cyrus_critic_evaluate")
        return self.q, self.qhat, self.loss

    def evaluate_noalloc(self, batch, seed: int, episode: int):
        """As evaluate, through cyrus_critic_evaluate_noalloc (per-row scratch in
        the library's static device array, not the workspace)."""
        ue, k, c, y, r = batch
        self._keep = batch
        b = cyrus_critic_batch(ctypes.cast(ue.data_ptr(), _i32p), ctypes.cast(k.data_ptr(), _i32p),
                               ctypes.cast(c.data_ptr(), _u8p), ctypes.cast(y.data_ptr(), _f32p),
                               ctypes.cast(r.data_ptr(), _f32p))
        _check(lib().cyrus_critic_evaluate_noalloc(self.handle, ctypes.byref(b), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                                   int(episode) & 0xFFFFFFFFFFFFFFFF, self.q.data_ptr(),
                                                   self.qhat.data_ptr(), self.loss.data_ptr(),
                                                   _stream_ptr(self.stream)), "cyrus_critic_evaluate_noalloc")
        return self.q, self.qhat, self.loss

    def close(self):
        if getattr(self, "handle", None):
            lib().cyrus_critic_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def critic_batch_to_device(batch, device: str = "cuda"):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in batch)
