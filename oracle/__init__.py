"""FP64 CPU oracle of the puncturing-codebook builder (ctypes wrapper).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package. It shares no code with the HIP
library: the arithmetic lives in ``cyrus_oracle.c`` (plain C, float64) and this
module only marshals numpy arrays. Configurations are duck-typed (any object
with num_ue, max_arrival, num_minislots, rb_per_unit, dims), so nothing here
imports the product package.

Parity status of each function (how it is pinned without trusting itself) is
recorded in the test files under tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cyrus_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libcyrus_oracle.so")
_lock = threading.Lock()
_lib = None

EXACT, BF16, FP8_E4M3 = 0, 1, 2
_PREC = {"exact": EXACT, "fp64": EXACT, "fp32": EXACT, "bf16": BF16, "fp8": FP8_E4M3}

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)


LARGEST_REMAINDER, HUNTINGTON_HILL = 0, 1
SOFTMAX_HEAD, GAUSSIAN_HEAD = 0, 1
_HEAD = {"softmax": SOFTMAX_HEAD, "gaussian": GAUSSIAN_HEAD}
_ROUNDING = {"lr": LARGEST_REMAINDER, "largest_remainder": LARGEST_REMAINDER, "hh": HUNTINGTON_HILL,
             "huntington_hill": HUNTINGTON_HILL}


class _Tree(ctypes.Structure):
    _fields_ = [("num_ue", ctypes.c_int32), ("max_arrival", ctypes.c_int32),
                ("num_minislots", ctypes.c_int32), ("rb_per_unit", ctypes.c_int32),
                ("rounding", ctypes.c_int32), ("head", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("tti", ctypes.c_uint64)]


class _CriticCfg(ctypes.Structure):
    _fields_ = [("num_ue", ctypes.c_int32), ("num_minislots", ctypes.c_int32), ("num_samples", ctypes.c_int32),
                ("discount", ctypes.c_double), ("entropy_coef", ctypes.c_double)]


class _Actor(ctypes.Structure):
    _fields_ = [("num_layers", ctypes.c_int32), ("dims", _i32p),
                ("w", ctypes.POINTER(_f32p)), ("b", ctypes.POINTER(_f32p)),
                ("precision", ctypes.c_int32), ("act_scale", _f64p),
                ("wq", ctypes.POINTER(_f64p))]


def compile_oracle(out_path: str = _LIB_PATH, src: str = _SRC, extra_flags=()) -> str:
    """Compile the C oracle with gcc (IEEE float64, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           *extra_flags, src, "-o", out_path, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out_path


def _load(path: str = _LIB_PATH):
    lib = ctypes.CDLL(path)
    lib.oracle_level_offset.restype = ctypes.c_int64
    lib.oracle_level_offset.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.oracle_num_nodes.restype = ctypes.c_int64
    lib.oracle_num_nodes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.oracle_round_bf16.restype = ctypes.c_double
    lib.oracle_round_bf16.argtypes = [ctypes.c_double]
    lib.oracle_round_e4m3.restype = ctypes.c_double
    lib.oracle_round_e4m3.argtypes = [ctypes.c_double]
    lib.oracle_e4m3_weight_scale.restype = ctypes.c_double
    lib.oracle_e4m3_weight_scale.argtypes = [_f32p, ctypes.c_int64]
    lib.oracle_quantize_weights.restype = None
    lib.oracle_quantize_weights.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int32, _f64p]
    lib.oracle_features.restype = None
    lib.oracle_features.argtypes = [ctypes.c_int32, _i32p, _i32p, _f32p, _i32p, ctypes.c_int32,
                                    ctypes.c_int32, _f64p]
    lib.oracle_mlp.restype = ctypes.c_int
    lib.oracle_mlp.argtypes = [ctypes.POINTER(_Actor), _f64p, _f64p, _f64p]
    lib.oracle_softmax.restype = None
    lib.oracle_softmax.argtypes = [ctypes.c_int32, _f64p, _f64p]
    lib.oracle_capped_scale.restype = ctypes.c_double
    lib.oracle_capped_scale.argtypes = [ctypes.c_int32, _f64p, _i32p, ctypes.c_int64, _f64p]
    lib.oracle_largest_remainder.restype = None
    lib.oracle_largest_remainder.argtypes = [ctypes.c_int32, _f64p, _i32p, ctypes.c_int64, _i32p]
    lib.oracle_margin.restype = ctypes.c_double
    lib.oracle_margin.argtypes = [ctypes.c_int32, _f64p, _i32p, ctypes.c_int64]
    lib.oracle_allocate.restype = ctypes.c_double
    lib.oracle_allocate.argtypes = [ctypes.c_int32, _f64p, _i32p, ctypes.c_int32, ctypes.c_int32,
                                    _i32p, _f64p]
    lib.oracle_allocate_rounding.restype = ctypes.c_double
    lib.oracle_allocate_rounding.argtypes = [ctypes.c_int32, _f64p, _i32p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, _i32p, _f64p]
    lib.oracle_huntington_hill.restype = None
    lib.oracle_huntington_hill.argtypes = [ctypes.c_int32, _f64p, _i32p, ctypes.c_int64, _i32p]
    lib.oracle_margin_hh.restype = ctypes.c_double
    lib.oracle_margin_hh.argtypes = [ctypes.c_int32, _f64p, _i32p, ctypes.c_int64, _i32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.oracle_normal.restype = ctypes.c_double
    lib.oracle_normal.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32]
    lib.oracle_gaussian_head.restype = None
    lib.oracle_gaussian_head.argtypes = [ctypes.c_int32, _f64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                         _f64p]
    lib.oracle_log_prob_tanh_gaussian.restype = ctypes.c_double
    lib.oracle_log_prob_tanh_gaussian.argtypes = [ctypes.c_int32, _f64p, _f64p]
    lib.oracle_sample_tanh_gaussian.restype = ctypes.c_double
    lib.oracle_sample_tanh_gaussian.argtypes = [ctypes.c_int32, _f64p, ctypes.c_uint64, ctypes.c_uint64,
                                                ctypes.c_int64, _f64p]
    lib.oracle_critic_evaluate.restype = ctypes.c_int
    lib.oracle_critic_evaluate.argtypes = [ctypes.POINTER(_CriticCfg)] + [ctypes.POINTER(_Actor)] * 5 + [
        _i32p, _i32p, _u8p, _f32p, _f32p, ctypes.c_uint64, ctypes.c_uint64, _f64p, _f64p, _f64p, _f64p]
    lib.oracle_build_tree.restype = ctypes.c_int
    lib.oracle_build_tree.argtypes = [ctypes.POINTER(_Tree), ctypes.POINTER(_Actor), _i32p, _i32p,
                                      _f32p, _u8p, _f64p, _f64p]
    lib.oracle_eval_conditioned.restype = ctypes.c_int
    lib.oracle_eval_conditioned.argtypes = [ctypes.POINTER(_Tree), ctypes.POINTER(_Actor), _i32p,
                                            _i32p, _f32p, _u8p, _i64p, ctypes.c_int64, _i32p, _f64p,
                                            _f64p]
    lib.oracle_rollout.restype = ctypes.c_int
    lib.oracle_rollout.argtypes = [ctypes.POINTER(_Tree), ctypes.POINTER(_Actor), _i32p, _i32p,
                                   _f32p, _i32p, ctypes.c_int32, _i32p, _f64p]
    lib.oracle_oru_assemble.restype = ctypes.c_int
    lib.oracle_oru_assemble.argtypes = [ctypes.POINTER(_Tree), ctypes.POINTER(_Actor), _i32p, _i32p, _f32p, _i32p,
                                        ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i32p]
    return lib


def lib():
    """The loaded oracle library; compiled from source if missing or stale."""
    global _lib
    with _lock:
        if _lib is None:
            stale = (not os.path.exists(_LIB_PATH)
                     or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC))
            if stale:
                compile_oracle()
            _lib = _load()
        return _lib


def _p(a: np.ndarray, ptype):
    return a.ctypes.data_as(ptype)


def _c(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class Actor:
    """Holds the ctypes view of an actor (weights stay referenced here)."""

    def __init__(self, weights, precision: str = "exact", act_scale=None, so=None):
        self.lib = so if so is not None else lib()
        self.precision = _PREC[precision]
        self.ws = [_c(w, np.float32) for w, _ in weights]
        self.bs = [_c(b, np.float32) for _, b in weights]
        dims = [self.ws[0].shape[1]] + [w.shape[0] for w in self.ws]
        self.dims = _c(dims, np.int32)
        n = len(self.ws)
        self._wp = (_f32p * n)(*[_p(w, _f32p) for w in self.ws])
        self._bp = (_f32p * n)(*[_p(b, _f32p) for b in self.bs])
        self.wq = None
        self._wqp = None
        if self.precision != EXACT:
            self.wq = []
            for w in self.ws:
                out = np.empty(w.size, dtype=np.float64)
                self.lib.oracle_quantize_weights(_p(w, _f32p), w.size, self.precision, _p(out, _f64p))
                self.wq.append(out)
            self._wqp = (_f64p * n)(*[_p(q, _f64p) for q in self.wq])
        self.act_scale = None if act_scale is None else _c(act_scale, np.float64)
        self.struct = _Actor(n, _p(self.dims, _i32p), self._wp, self._bp, self.precision,
                             None if self.act_scale is None else _p(self.act_scale, _f64p),
                             self._wqp)


def _tree(cfg, seed: int = 0, tti: int = 0) -> _Tree:
    return _Tree(cfg.num_ue, cfg.max_arrival, cfg.num_minislots, cfg.rb_per_unit,
                 _ROUNDING[getattr(cfg, "rounding", "lr")], _HEAD[getattr(cfg, "head", "softmax")],
                 int(seed) & 0xFFFFFFFFFFFFFFFF, int(tti) & 0xFFFFFFFFFFFFFFFF)


def _ue_arrays(ue):
    return _c(ue.rb, np.int32), _c(ue.mcs, np.int32), _c(ue.sinr_db, np.float32)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


# ----------------------------------------------------------------- tree shape

def level_offset(K: int, tau: int) -> int:
    return int(lib().oracle_level_offset(K, tau))


def num_nodes(K: int, M: int) -> int:
    return int(lib().oracle_num_nodes(K, M))


# ------------------------------------------------------------- number formats

def round_bf16(v: float) -> float:
    return float(lib().oracle_round_bf16(float(v)))


def round_e4m3(v: float) -> float:
    return float(lib().oracle_round_e4m3(float(v)))


def e4m3_weight_scale(w) -> float:
    w = _c(w, np.float32).ravel()
    return float(lib().oracle_e4m3_weight_scale(_p(w, _f32p), w.size))


# ---------------------------------------------------------------- node steps

def features(ue, c, tau: int, k: int) -> np.ndarray:
    rb, mcs, sinr = _ue_arrays(ue)
    E = rb.shape[0]
    c = _c(c, np.int32)
    x = np.empty(4 * E + 2, dtype=np.float64)
    lib().oracle_features(E, _p(rb, _i32p), _p(mcs, _i32p), _p(sinr, _f32p), _p(c, _i32p), tau, k,
                          _p(x, _f64p))
    return x


def mlp(weights, x, precision: str = "exact", act_scale=None, actor: Actor | None = None,
        amax: np.ndarray | None = None) -> np.ndarray:
    f = actor or Actor(weights, precision, act_scale)
    x = _c(x, np.float64)
    z = np.empty(int(f.dims[-1]), dtype=np.float64)
    _check(f.lib.oracle_mlp(ctypes.byref(f.struct), _p(x, _f64p), _p(z, _f64p),
                            None if amax is None else _p(amax, _f64p)), "mlp")
    return z


def softmax(z) -> np.ndarray:
    z = _c(z, np.float64)
    p = np.empty_like(z)
    lib().oracle_softmax(z.size, _p(z, _f64p), _p(p, _f64p))
    return p


def capped_scale(p, R, T: int):
    """Returns (x, s): the capped proportional split of T and its multiplier."""
    p = _c(p, np.float64)
    R = _c(R, np.int32)
    x = np.empty_like(p)
    s = lib().oracle_capped_scale(p.size, _p(p, _f64p), _p(R, _i32p), int(T), _p(x, _f64p))
    return x, float(s)


def largest_remainder(x, R, T: int) -> np.ndarray:
    x = _c(x, np.float64)
    R = _c(R, np.int32)
    a = np.empty(x.size, dtype=np.int32)
    lib().oracle_largest_remainder(x.size, _p(x, _f64p), _p(R, _i32p), int(T), _p(a, _i32p))
    return a


def huntington_hill(x, R, T: int) -> np.ndarray:
    x = _c(x, np.float64)
    R = _c(R, np.int32)
    a = np.empty(x.size, dtype=np.int32)
    lib().oracle_huntington_hill(x.size, _p(x, _f64p), _p(R, _i32p), int(T), _p(a, _i32p))
    return a


def margin_hh(x, R, T: int, a) -> float:
    """Max-norm distance of the shares x from the nearest change of the
    Huntington-Hill allocation a."""
    x = _c(x, np.float64)
    R = _c(R, np.int32)
    a = _c(a, np.int32)
    return float(lib().oracle_margin_hh(x.size, _p(x, _f64p), _p(R, _i32p), int(T), _p(a, _i32p)))


def margin(x, R, T: int) -> float:
    """Max-norm distance of the shares x from the nearest change of their
    largest-remainder allocation."""
    x = _c(x, np.float64)
    R = _c(R, np.int32)
    return float(lib().oracle_margin(x.size, _p(x, _f64p), _p(R, _i32p), int(T)))


def allocate(z, R, U: int, k: int, rounding: str = "lr"):
    """Returns (a, margin, x) for one node's logits."""
    z = _c(z, np.float64)
    R = _c(R, np.int32)
    a = np.empty(z.size, dtype=np.int32)
    x = np.empty(z.size, dtype=np.float64)
    m = lib().oracle_allocate_rounding(z.size, _p(z, _f64p), _p(R, _i32p), U, k, _ROUNDING[rounding],
                                       _p(a, _i32p), _p(x, _f64p))
    return a, float(m), x


# ---------------------------------------------------------------- Gaussian head

def philox4x32_10(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(c.ctypes.data_as(_u32p), k.ctypes.data_as(_u32p), out.ctypes.data_as(_u32p))
    return out


def normal(seed: int, tti: int, node: int, e: int) -> float:
    return float(lib().oracle_normal(int(seed) & 0xFFFFFFFFFFFFFFFF, int(tti) & 0xFFFFFFFFFFFFFFFF, int(node), int(e)))


def gaussian_head(out, seed: int, tti: int, node: int) -> np.ndarray:
    """Log-shares z (E) of one node from the actor's 2E outputs (mu, log sigma)."""
    out = _c(out, np.float64)
    E = out.size // 2
    z = np.zeros(E, dtype=np.float64)
    lib().oracle_gaussian_head(E, _p(out, _f64p), int(seed) & 0xFFFFFFFFFFFFFFFF, int(tti) & 0xFFFFFFFFFFFFFFFF,
                               int(node), _p(z, _f64p))
    return z


def log_prob_tanh_gaussian(out, u) -> float:
    """log pi of the action (1 + tanh u) / 2 under the actor outputs (mu, log sigma)."""
    out = _c(out, np.float64)
    u = _c(u, np.float64)
    return float(lib().oracle_log_prob_tanh_gaussian(u.size, _p(out, _f64p), _p(u, _f64p)))


def sample_tanh_gaussian(out, seed: int, tti: int, node: int):
    """(y, log pi(y)): the policy's action for actor outputs (mu, log sigma)."""
    out = _c(out, np.float64)
    E = out.size // 2
    y = np.zeros(E, dtype=np.float64)
    lp = lib().oracle_sample_tanh_gaussian(E, _p(out, _f64p), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                           int(tti) & 0xFFFFFFFFFFFFFFFF, int(node), _p(y, _f64p))
    return y, float(lp)


def critic_evaluate(E: int, M: int, actor_w, q_w, qt_w, ue, k, c, y, r, seed: int, episode: int,
                    discount: float, entropy_coef: float):
    """Critic pass over H buffer samples (Eqs. (3), (4)). ue [H,3E] i32 (rb, mcs,
    sinr bits), k [H,M], c [H,M,E] u8, y [H,M,E] f32, r [H] f32; q_w and qt_w are
    pairs of critic weight lists. Returns (q [2,H,M], qhat [H,M], logpi [H,M],
    loss [2])."""
    ue = _c(ue, np.int32)
    H = ue.shape[0]
    k = _c(k, np.int32)
    c = _c(c, np.uint8)
    y = _c(y, np.float32)
    r = _c(r, np.float32)
    nets = [Actor(actor_w)] + [Actor(w) for w in q_w] + [Actor(w) for w in qt_w]
    cfg = _CriticCfg(E, M, H, float(discount), float(entropy_coef))
    q = np.zeros((2, H, M), dtype=np.float64)
    qhat = np.zeros((H, M), dtype=np.float64)
    lp = np.zeros((H, M), dtype=np.float64)
    loss = np.zeros(2, dtype=np.float64)
    _check(lib().oracle_critic_evaluate(ctypes.byref(cfg), *[ctypes.byref(n.struct) for n in nets], _p(ue, _i32p),
                                        _p(k, _i32p), _p(c, _u8p), _p(y, _f32p), _p(r, _f32p),
                                        int(seed) & 0xFFFFFFFFFFFFFFFF, int(episode) & 0xFFFFFFFFFFFFFFFF,
                                        _p(q, _f64p), _p(qhat, _f64p), _p(lp, _f64p), _p(loss, _f64p)),
           "critic_evaluate")
    return q, qhat, lp, loss


# ---------------------------------------------------------------------- trees

def build_tree(cfg, weights, ue, precision: str = "exact", act_scale=None, actor: Actor | None = None,
               seed: int = 0, tti: int = 0):
    """Free-running FP64 codebook. Returns (alloc [nodes,E] u8, logits [nodes,E]
    f64, margin [nodes] f64)."""
    f = actor or Actor(weights, precision, act_scale)
    rb, mcs, sinr = _ue_arrays(ue)
    n, E = cfg.num_nodes, cfg.num_ue
    alloc = np.zeros((n, E), dtype=np.uint8)
    logits = np.zeros((n, E), dtype=np.float64)
    marg = np.zeros(n, dtype=np.float64)
    t = _tree(cfg, seed, tti)
    _check(f.lib.oracle_build_tree(ctypes.byref(t), ctypes.byref(f.struct), _p(rb, _i32p), _p(mcs, _i32p),
                                   _p(sinr, _f32p), _p(alloc, _u8p), _p(logits, _f64p), _p(marg, _f64p)),
           "build_tree")
    return alloc, logits, marg


def eval_conditioned(cfg, weights, ue, given_alloc, nodes=None, precision: str = "exact",
                     act_scale=None, actor: Actor | None = None, seed: int = 0, tti: int = 0):
    """Recompute the listed nodes (all if None) from the state their ancestors
    reach under `given_alloc`. Returns (alloc [n,E] i32, logits [n,E], margin [n])."""
    f = actor or Actor(weights, precision, act_scale)
    rb, mcs, sinr = _ue_arrays(ue)
    E = cfg.num_ue
    given = _c(given_alloc, np.uint8)
    if given.shape != (cfg.num_nodes, E):
        raise ValueError(f"given_alloc shape {given.shape} != {(cfg.num_nodes, E)}")
    ids = _c(np.arange(cfg.num_nodes) if nodes is None else nodes, np.int64)
    n = ids.size
    alloc = np.zeros((n, E), dtype=np.int32)
    logits = np.zeros((n, E), dtype=np.float64)
    marg = np.zeros(n, dtype=np.float64)
    t = _tree(cfg, seed, tti)
    _check(f.lib.oracle_eval_conditioned(ctypes.byref(t), ctypes.byref(f.struct), _p(rb, _i32p),
                                         _p(mcs, _i32p), _p(sinr, _f32p), _p(given, _u8p), _p(ids, _i64p),
                                         n, _p(alloc, _i32p), _p(logits, _f64p), _p(marg, _f64p)),
           "eval_conditioned")
    return alloc, logits, marg


def rollout(cfg, weights, ue, seq, precision: str = "exact", act_scale=None,
            actor: Actor | None = None, amax: np.ndarray | None = None, seed: int = 0, tti: int = 0) -> np.ndarray:
    f = actor or Actor(weights, precision, act_scale)
    rb, mcs, sinr = _ue_arrays(ue)
    seq = _c(seq, np.int32)
    out = np.zeros((seq.size, cfg.num_ue), dtype=np.int32)
    t = _tree(cfg, seed, tti)
    _check(f.lib.oracle_rollout(ctypes.byref(t), ctypes.byref(f.struct), _p(rb, _i32p), _p(mcs, _i32p),
                                _p(sinr, _f32p), _p(seq, _i32p), seq.size, _p(out, _i32p),
                                None if amax is None else _p(amax, _f64p)), "rollout")
    return out


def node_index(K: int, seq) -> int:
    """BFS index of the node reached by arrival prefix seq = (k_1..k_tau)."""
    tau = len(seq)
    i = 0
    for k in seq:
        i = i * (K + 1) + int(k)
    return level_offset(K, tau) + i


def oru_assemble(cfg, weights, ue, raw, carry_in: int = 0, actor: Actor | None = None, seed: int = 0,
                 tti: int = 0):
    """Controller capping/buffering plus Alg. 3: returns (served [len], Y [len,E], carry_out)."""
    f = actor or Actor(weights)
    rb, mcs, sinr = _ue_arrays(ue)
    raw = _c(raw, np.int32)
    served = np.zeros(raw.size, dtype=np.int32)
    y = np.zeros((raw.size, cfg.num_ue), dtype=np.int32)
    co = ctypes.c_int32()
    t = _tree(cfg, seed, tti)
    _check(f.lib.oracle_oru_assemble(ctypes.byref(t), ctypes.byref(f.struct), _p(rb, _i32p), _p(mcs, _i32p),
                                     _p(sinr, _f32p), _p(raw, _i32p), raw.size, int(carry_in), _p(served, _i32p),
                                     _p(y, _i32p), ctypes.byref(co)), "oru_assemble")
    return served, y, co.value
