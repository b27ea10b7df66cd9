"""Comparison of a codebook from the HIP library with the FP64 oracle.

Conditioned mode (the gate): every node is recomputed by the oracle from the
state its ancestors reach under the GPU's own codebook, so one disagreement
cannot spread. The oracle's decision margin of a node is the max-norm distance
of its float64 shares from the nearest share vector that rounds differently.

- FP32 (the exact rule): a node may disagree only if that margin is below
  1e-6. Such boundary cases are counted and reported.
- Reduced precision (against the oracle run in the same precision): a node
  may disagree only if the margin is below what the GPU's arithmetic can move
  the shares there. Its logits differ from the oracle's by dz (measured per
  node); each share x_e = s p_e then moves by at most x_e (e^(2 dz) - 1) <=
  4 dz T for dz <= 1/2, plus the FP32 rounding of the exponentials, the E-term
  sum, the division and the product, (E + 4) eps relative. The bound used is
  twice that: B = T (8 dz + 4 (E + 4) eps32).

Free-running mode: the oracle builds its own tree; every node where the two
trees differ must lie in the subtree of a conditioned-mode disagreement.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle

EPS32 = 2.0 ** -24
BOUNDARY = 1e-6


def share_bound(T: int, E: int, dz: float) -> float:
    """Twice the max-norm distance the GPU's FP32 shares can sit from the
    oracle's at a node of demand T whose logits differ by at most dz."""
    assert dz <= 0.5, f"logit error {dz} beyond the range of the bound"
    return T * (8.0 * dz + 4.0 * (E + 4) * EPS32)


@dataclasses.dataclass
class ParityReport:
    nodes: int
    evals: int
    cond_mismatch: int
    cond_unexplained: int
    boundary_below_1e6: int
    boundary_above_1e6: int
    max_logit_err: float
    free_mismatch: int
    free_unexplained: int
    min_margin_mismatch: float
    disagreement_rate_cond: float
    disagreement_rate_free: float

    def as_dict(self):
        return dataclasses.asdict(self)

    def check(self, tag: str, exact: bool):
        """The gate: no unexplained disagreement in either mode; with `exact`
        (FP32 against the FP64 oracle) every disagreement lies within 1e-6 of
        a rounding boundary."""
        print(f"[parity] {tag}: {self.as_dict()}", flush=True)
        assert self.cond_unexplained == 0, f"{tag}: {self.cond_unexplained} unexplained conditioned mismatches"
        assert self.free_unexplained == 0, f"{tag}: {self.free_unexplained} unexplained free-running mismatches"
        if exact:
            assert self.boundary_above_1e6 == 0, (
                f"{tag}: {self.boundary_above_1e6} disagreements with a margin above {BOUNDARY}")


def level_of(cfg, node: int) -> int:
    tau = 0
    while oracle.level_offset(cfg.max_arrival, tau + 1) <= node:
        tau += 1
    return tau


def ancestors(cfg, node: int):
    """Strict ancestors of a node (excluding the root)."""
    K = cfg.max_arrival
    tau = level_of(cfg, node)
    i = node - oracle.level_offset(K, tau)
    out = []
    for lev in range(tau - 1, 0, -1):
        i //= (K + 1)
        out.append(oracle.level_offset(K, lev) + i)
    return out


def demand(cfg, ue, node: int) -> int:
    K = cfg.max_arrival
    tau = level_of(cfg, node)
    if tau == 0:
        return 0
    k = (node - oracle.level_offset(K, tau)) % (K + 1)
    return min(cfg.rb_per_unit * k, int(np.asarray(ue.rb).sum()))


def compare(cfg, weights, ue, gpu_alloc, gpu_logits, nodes=None, actor=None, precision="exact",
            act_scale=None, logit_tol=None, free_running=True, seed=0, tti=0) -> ParityReport:
    """Compare a GPU codebook and its exported logits with the oracle.
    `nodes` restricts the conditioned check to a sample (free-running is then
    skipped). A disagreement is a boundary case below 1e-6, else explained if
    its margin lies below share_bound(T, E, dz) for the node's measured logit
    error dz, else unexplained."""
    actor = actor or oracle.Actor(weights, precision, act_scale)
    ids = np.arange(cfg.num_nodes) if nodes is None else np.asarray(nodes, dtype=np.int64)
    c_alloc, c_logits, c_margin = oracle.eval_conditioned(cfg, weights, ue, gpu_alloc, ids, actor=actor, seed=seed,
                                                          tti=tti)
    g = np.asarray(gpu_alloc)[ids].astype(np.int32)
    mism = np.nonzero((c_alloc != g).any(axis=1))[0]
    dz = np.abs(np.asarray(gpu_logits, np.float64)[ids] - c_logits).max(axis=1)
    max_dz = float(dz.max()) if dz.size else 0.0
    if logit_tol is not None:
        assert max_dz <= logit_tol, f"max logit error {max_dz:.3e} above {logit_tol:.3e}"
    unexplained = 0
    below, above = 0, 0
    min_m = np.inf
    for j in mism:
        node = int(ids[j])
        m = c_margin[j]
        min_m = min(min_m, m)
        if m < BOUNDARY:
            below += 1
        elif m < share_bound(demand(cfg, ue, node), cfg.num_ue, dz[j]):
            above += 1
        else:
            unexplained += 1
    K = cfg.max_arrival
    evals_mask = np.array([level_of(cfg, int(n)) > 0 and (int(n) - oracle.level_offset(K, level_of(cfg, int(n))))
                           % (K + 1) != 0 for n in ids]) if nodes is not None else None
    n_evals = int(evals_mask.sum()) if evals_mask is not None else cfg.num_evals
    free_m, free_bad = 0, 0
    if free_running and nodes is None:
        f_alloc, _, _ = oracle.build_tree(cfg, weights, ue, actor=actor, seed=seed, tti=tti)
        diff = np.nonzero((f_alloc != np.asarray(gpu_alloc)).any(axis=1))[0]
        free_m = int(diff.size)
        cond_set = set(int(ids[j]) for j in mism)
        for node in diff:
            node = int(node)
            if node in cond_set or any(a in cond_set for a in ancestors(cfg, node)):
                continue
            free_bad += 1
    return ParityReport(nodes=int(ids.size), evals=n_evals, cond_mismatch=int(mism.size),
                        cond_unexplained=unexplained, boundary_below_1e6=below, boundary_above_1e6=above,
                        max_logit_err=max_dz, free_mismatch=free_m, free_unexplained=free_bad,
                        min_margin_mismatch=float(min_m),
                        disagreement_rate_cond=mism.size / max(n_evals, 1),
                        disagreement_rate_free=free_m / max(n_evals, 1))


def check_invariants(cfg, ue, alloc):
    """Sum, caps, zero branch and monotone state at every node."""
    K, M, U, E = cfg.max_arrival, cfg.num_minislots, cfg.rb_per_unit, cfg.num_ue
    alloc = np.asarray(alloc).astype(np.int64)
    R = np.asarray(ue.rb, np.int64)
    assert not alloc[0].any(), "root must puncture nothing"
    for tau in range(1, M + 1):
        off, poff = oracle.level_offset(K, tau), oracle.level_offset(K, tau - 1)
        width = (K + 1) ** tau
        a = alloc[off:off + width]
        k = np.arange(width) % (K + 1)
        T = np.minimum(U * k, R.sum())
        assert np.array_equal(a.sum(axis=1), T), f"level {tau}: sums differ from min(Uk, sum R)"
        assert np.all(a <= R[None, :]), f"level {tau}: an allocation exceeds its cap"
        assert not a[k == 0].any(), f"level {tau}: a k = 0 node punctures"
