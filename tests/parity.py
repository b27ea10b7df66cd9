"""Comparison of a codebook from the HIP library with the FP64 oracle.

Conditioned mode (the gate): every node is recomputed by the oracle from the
state its ancestors reach under the GPU's own codebook, so one disagreement
cannot spread. A node may disagree only if the oracle's float64 decision
margin is below the perturbation the GPU's arithmetic can cause there:

  the GPU logits differ from the oracle's by dz (measured per node), which
  moves every share x_e = T p_e / sum p by at most T (4 dz + 8 eps) to first
  order (softmax ratio plus FP32 rounding of exp, sum and division), so a
  remainder gap can close by twice that. The bound used is
  B = 2 * T * (8 dz + 16 eps32), a further factor two of slack.

Free-running mode: the oracle builds its own tree; every node where the two
trees differ must lie in the subtree of a conditioned-mode disagreement.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle

EPS32 = 2.0 ** -24


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


def compare(cfg, weights, ue, gpu_alloc, gpu_logits=None, nodes=None, actor=None, precision="exact",
            act_scale=None, logit_tol=None, free_running=True, margin_slack=1.0, dz_floor=0.0, seed=0,
            tti=0) -> ParityReport:
    """Compare a GPU codebook with the oracle. `nodes` restricts the
    conditioned check to a sample (free-running is then skipped). Without GPU
    logits, `dz_floor` stands in for the per-node logit error (a tolerance
    established by the tests that do export logits)."""
    actor = actor or oracle.Actor(weights, precision, act_scale)
    ids = np.arange(cfg.num_nodes) if nodes is None else np.asarray(nodes, dtype=np.int64)
    c_alloc, c_logits, c_margin = oracle.eval_conditioned(cfg, weights, ue, gpu_alloc, ids, actor=actor, seed=seed,
                                                          tti=tti)
    g = np.asarray(gpu_alloc)[ids].astype(np.int32)
    mism = np.nonzero((c_alloc != g).any(axis=1))[0]
    if gpu_logits is not None:
        dz = np.abs(np.asarray(gpu_logits, np.float64)[ids] - c_logits).max(axis=1)
    else:
        dz = np.zeros(ids.size)
    dz = np.maximum(dz, dz_floor)
    max_dz = float(dz.max()) if dz.size else 0.0
    if logit_tol is not None:
        assert max_dz <= logit_tol, f"max logit error {max_dz:.3e} above {logit_tol:.3e}"
    unexplained = 0
    below, above = 0, 0
    min_m = np.inf
    for j in mism:
        node = int(ids[j])
        T = demand(cfg, ue, node)
        bound = margin_slack * 2.0 * T * (8.0 * dz[j] + 16.0 * EPS32)
        m = c_margin[j]
        min_m = min(min_m, m)
        if m < 1e-6:
            below += 1
        elif m < bound:
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
