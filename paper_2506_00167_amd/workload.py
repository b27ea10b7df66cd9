"""Seeded synthetic inputs for the puncturing-codebook builder.

This module only draws numbers: actor weights, per-UE scheduling state and the
named tree shapes. It holds none of the method's arithmetic, so both the HIP
path and the FP64 oracle can consume what it produces without sharing code.

Input recipe (the paper's simulator and trained actor are not available, so
seeded draws stand in for them):

* eMBB scheduling vector s(t) (Sec. III-A): per UE an RB count R_e ~ U{8..32};
  the per-UE channel features are MCS_e ~ U{0..27} and SINR_e ~ N(15, 5) dB,
  drawn in float64 and rounded to float32 (the value both paths consume).
* Actor weights f_a (Sec. V-B): a ReLU MLP, Xavier-uniform weights
  U(+-sqrt(6/(fan_in+fan_out))) and biases U(+-1/sqrt(fan_in)), drawn in
  float64 and rounded to float32. Row-major [out][in].
* URLLC arrival alphabet {0..K} per mini-slot, K = floor(N/L) (Sec. IV-A).
"""
from __future__ import annotations

import dataclasses
from typing import Sequence, List, Tuple

import numpy as np

PRECISIONS = ("fp32", "bf16", "fp8")


@dataclasses.dataclass(frozen=True)
class TreeConfig:
    """Shape of one codebook tree and its actor network.

    num_ue        E, eMBB UEs per cell.
    max_arrival   K = floor(N/L), largest URLLC arrival count per mini-slot.
    num_minislots M, mini-slots per slot (7 in NR).
    rb_per_unit   U, RBs one URLLC arrival punctures.
    hidden        hidden widths of the actor MLP.
    precision     arithmetic of the layer GEMMs: fp32, bf16 or fp8 (e4m3).
    rounding      integer step of the enforcer: "lr" (largest remainder) or
                  "hh" (Huntington-Hill).
    head          policy head: "softmax" (E logits) or "gaussian" (2E outputs,
                  means and log standard deviations, sampled per node).
    """

    num_ue: int
    max_arrival: int
    num_minislots: int = 7
    rb_per_unit: int = 2
    hidden: Tuple[int, ...] = (256, 256)
    precision: str = "fp32"
    rounding: str = "lr"
    head: str = "softmax"

    @property
    def d_in(self) -> int:
        return 4 * self.num_ue + 2

    @property
    def dims(self) -> Tuple[int, ...]:
        return (self.d_in,) + tuple(self.hidden) + (self.num_ue * (2 if self.head == "gaussian" else 1),)

    @property
    def num_nodes(self) -> int:
        k1 = self.max_arrival + 1
        return (k1 ** (self.num_minislots + 1) - 1) // self.max_arrival

    @property
    def num_evals(self) -> int:
        return (self.max_arrival + 1) ** self.num_minislots - 1

    @property
    def macs_per_eval(self) -> int:
        d = self.dims
        return sum(d[i] * d[i + 1] for i in range(len(d) - 1))

    @property
    def flops_per_codebook(self) -> int:
        return 2 * self.macs_per_eval * self.num_evals

    @property
    def flops_per_codebook_folded(self) -> int:
        """FLOPs when the first layer's static inputs (R, MCS, SINR: 3E of them,
        the same at every node) are multiplied once per codebook and each
        evaluation multiplies only its own E + 2 inputs (c, tau, k)."""
        d = self.dims
        static = 3 * self.num_ue
        per_eval = (d[0] - static) * d[1] + sum(d[i] * d[i + 1] for i in range(1, len(d) - 1))
        return 2 * (per_eval * self.num_evals + static * d[1])

    def with_precision(self, precision: str) -> "TreeConfig":
        return dataclasses.replace(self, precision=precision)

    def with_rounding(self, rounding: str) -> "TreeConfig":
        return dataclasses.replace(self, rounding=rounding)

    def with_head(self, head: str) -> "TreeConfig":
        return dataclasses.replace(self, head=head)


# Named workloads. The first is small enough for the oracle to finish in well
# under a second; the second is the single-codebook latency workload.
TINY = TreeConfig(num_ue=4, max_arrival=2, hidden=(256, 256))
TREE_E8K3 = TreeConfig(num_ue=8, max_arrival=3, hidden=(256, 256))
STRESS_E16K4 = TreeConfig(num_ue=16, max_arrival=4, hidden=(512, 512, 512), precision="fp8")
# The paper's own codebook shape: depth 1, E = 10, K = floor(780/300) = 2,
# one hidden layer of 128 neurons (Sec. VI, case-study parameters).
PAPER_DEPTH1 = TreeConfig(num_ue=10, max_arrival=2, num_minislots=1, hidden=(128,))

WORKLOADS = {
    "tiny-e4k2": TINY,
    "tree-e8k3": TREE_E8K3,
    "stress-e16k4": STRESS_E16K4,
    "paper-depth1": PAPER_DEPTH1,
}

WEIGHT_SEEDS = {"tiny-e4k2": 1, "tree-e8k3": 2, "stress-e16k4": 200000, "paper-depth1": 4}
CALIBRATION_SEED = 3
UE_SEED_BASE = 1_000_000


def make_weights(cfg: TreeConfig, seed: int) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Xavier-uniform float32 weights [out][in] and uniform biases per layer."""
    return make_net_weights(cfg.dims, seed)


def make_net_weights(d: Sequence[int], seed: int) -> List[Tuple[np.ndarray, np.ndarray]]:
    """The same recipe for any layer widths d[0] -> d[1] -> ... -> d[-1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    layers = []
    for i in range(len(d) - 1):
        fan_in, fan_out = d[i], d[i + 1]
        lim_w = np.sqrt(6.0 / (fan_in + fan_out))
        lim_b = 1.0 / np.sqrt(fan_in)
        w = rng.uniform(-lim_w, lim_w, size=(fan_out, fan_in)).astype(np.float32)
        b = rng.uniform(-lim_b, lim_b, size=(fan_out,)).astype(np.float32)
        layers.append((np.ascontiguousarray(w), np.ascontiguousarray(b)))
    return layers


@dataclasses.dataclass
class UEState:
    """Per-UE scheduling state of one TTI: RBs, MCS index and SINR (dB)."""

    rb: np.ndarray  # int32 [E]
    mcs: np.ndarray  # int32 [E]
    sinr_db: np.ndarray  # float32 [E]

    @property
    def num_ue(self) -> int:
        return int(self.rb.shape[0])


def make_ue_state(num_ue: int, seed: int) -> UEState:
    rng = np.random.Generator(np.random.PCG64(seed))
    rb = rng.integers(8, 33, size=num_ue).astype(np.int32)
    mcs = rng.integers(0, 28, size=num_ue).astype(np.int32)
    sinr = rng.normal(15.0, 5.0, size=num_ue).astype(np.float32)
    return UEState(rb=rb, mcs=mcs, sinr_db=sinr)


def make_ue_state_edge(num_ue: int, seed: int, max_rb: int = 4) -> UEState:
    """UE state with tiny RB counts (including unscheduled UEs, R_e = 0) so that
    per-UE caps and the demand-above-capacity case are exercised."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rb = rng.integers(0, max_rb + 1, size=num_ue).astype(np.int32)
    mcs = rng.integers(0, 28, size=num_ue).astype(np.int32)
    sinr = rng.normal(15.0, 5.0, size=num_ue).astype(np.float32)
    return UEState(rb=rb, mcs=mcs, sinr_db=sinr)


def ue_seed(i: int) -> int:
    return UE_SEED_BASE + i


@dataclasses.dataclass(frozen=True)
class CriticConfig:
    """The Near-RT RIC's critic pass (Sec. IV-B): H buffer samples of M steps
    for E UEs; an actor with the Gaussian head (2E outputs) and four critics
    (Q1, Q2 and their targets) of the given hidden widths on [state, y]."""

    num_ue: int = 8
    max_arrival: int = 3
    num_minislots: int = 7
    num_samples: int = 256
    rb_per_unit: int = 2
    actor_hidden: Tuple[int, ...] = (256, 256)
    critic_hidden: Tuple[int, ...] = (256, 256)
    discount: float = 0.99
    entropy_coef: float = 0.2

    @property
    def actor_dims(self) -> Tuple[int, ...]:
        return (4 * self.num_ue + 2,) + tuple(self.actor_hidden) + (2 * self.num_ue,)

    @property
    def critic_dims(self) -> Tuple[int, ...]:
        return (5 * self.num_ue + 2,) + tuple(self.critic_hidden) + (1,)

    @property
    def rows(self) -> int:
        return self.num_samples * self.num_minislots

    @property
    def flops(self) -> int:
        """Algorithmic FLOPs of one pass: two critics on every row; the actor
        and two target critics on every row but the last step of a sample."""
        mac = lambda d: sum(d[i] * d[i + 1] for i in range(len(d) - 1))  # noqa: E731
        H, M = self.num_samples, self.num_minislots
        return 2 * (2 * H * M * mac(self.critic_dims) + H * (M - 1) * (mac(self.actor_dims) + 2 * mac(self.critic_dims)))


CRITIC_RIC = CriticConfig()


def make_critic_weights(cfg: CriticConfig, seed: int):
    """(actor, [Q1, Q2], [Qtarg1, Qtarg2]) weight lists."""
    actor = make_net_weights(cfg.actor_dims, seed)
    q = [make_net_weights(cfg.critic_dims, seed + 1 + i) for i in range(2)]
    qt = [make_net_weights(cfg.critic_dims, seed + 3 + i) for i in range(2)]
    return actor, q, qt


def make_critic_batch(cfg: CriticConfig, seed: int):
    """H synthetic buffer samples: UE state per sample (ue [H,3E] int32: rb,
    mcs, sinr bits), arrivals k [H,M] in 0..K, stored actions y [H,M,E] in
    (0,1), carried punctured RBs c [H,M,E] (0 at step 1, then the running sum of
    floor(y * min(R, U k)) of the earlier steps, within 8 bits) and rewards r [H]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H, M, E = cfg.num_samples, cfg.num_minislots, cfg.num_ue
    ue = np.zeros((H, 3 * E), dtype=np.int32)
    for h in range(H):
        st = make_ue_state(E, int(rng.integers(0, 2**31)))
        ue[h, :E] = st.rb
        ue[h, E:2 * E] = st.mcs
        ue[h, 2 * E:] = st.sinr_db.view(np.int32)
    k = rng.integers(0, cfg.max_arrival + 1, size=(H, M)).astype(np.int32)
    y = rng.uniform(0.01, 0.99, size=(H, M, E)).astype(np.float32)
    c = np.zeros((H, M, E), dtype=np.uint8)
    for tau in range(1, M):
        cap = np.minimum(ue[:, None, :E], (cfg.rb_per_unit * k[:, tau - 1])[:, None, None])[:, 0, :]
        step = np.floor(y[:, tau - 1, :] * cap).astype(np.int64)
        c[:, tau, :] = np.minimum(c[:, tau - 1, :].astype(np.int64) + step, 255).astype(np.uint8)
    r = rng.normal(0.0, 1.0, size=H).astype(np.float32)
    return ue, k, c, y, r


def serving_cell_configs(num_cells: int = 64, seed: int = 424242) -> List[Tuple[TreeConfig, int]]:
    """Per-cell shapes of the serving mix: E ~ U{4..16}, K ~ U{2,3,4}, two hidden
    layers of 256 or 512, bf16. Returns (config, weight seed) per cell."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cells = []
    for j in range(num_cells):
        e = int(rng.integers(4, 17))
        k = int(rng.choice([2, 3, 4]))
        h = int(rng.choice([256, 512]))
        cells.append((TreeConfig(num_ue=e, max_arrival=k, hidden=(h, h), precision="bf16"), 100_000 + j))
    return cells


def poisson_arrivals(rate_per_s: float, count: int, seed: int = 424242) -> np.ndarray:
    """Arrival times (s) of a Poisson request stream."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def random_sequences(cfg: TreeConfig, count: int, seed: int) -> np.ndarray:
    """Random arrival sequences k_1..k_M, each k in {0..K}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, cfg.max_arrival + 1, size=(count, cfg.num_minislots)).astype(np.int32)


def sample_nodes(cfg: TreeConfig, count: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(cfg.num_nodes, size=min(count, cfg.num_nodes), replace=False)).astype(np.int64)
