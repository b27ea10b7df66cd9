"""Pins of the oracle's Gaussian policy head (Sec. IV-B: per-UE means and
standard deviations, a reparameterised sample, tanh), independent of its own
code:

- Philox4x32-10 against the generator authors' known-answer vectors;
- the normal draws against N(0, 1) (Kolmogorov-Smirnov, moments, and no
  correlation between neighbouring counters);
- the head's log-shares against numpy's tanh on the same draws, the
  standard-deviation clamp, and the small-sigma limit;
- a tree with the Gaussian head equals sequential roll-outs of every arrival
  sequence (the per-node counters agree), depends on the TTI, and keeps the
  allocation invariants.
"""
import itertools
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2506_00167_amd import workload as wl
from tests import parity
from tests import test_oracle_tree as tt

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(v, 16) for v in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert oracle.philox4x32_10(ctr, key).tolist() == want


def test_normal_is_standard():
    draws = np.array([oracle.normal(7, 11, node, e) for node in range(2500) for e in range(8)])
    assert abs(draws.mean()) < 0.03 and abs(draws.var() - 1.0) < 0.04
    assert stats.kstest(draws, "norm").pvalue > 1e-3
    a = draws.reshape(2500, 8)
    assert abs(np.corrcoef(a[:, 0], a[:, 1])[0, 1]) < 0.06       # neighbouring UEs
    assert abs(np.corrcoef(a[:-1, 3], a[1:, 3])[0, 1]) < 0.06     # neighbouring nodes


def test_normal_depends_on_every_key_part():
    base = oracle.normal(1, 2, 3, 4)
    for args in [(2, 2, 3, 4), (1, 3, 3, 4), (1, 2, 4, 4), (1, 2, 3, 5), (1, 2 + (1 << 32), 3, 4),
                 (1 + (1 << 32), 2, 3, 4)]:
        assert oracle.normal(*args) != base, args


def test_head_matches_tanh_on_the_same_draws():
    rng = np.random.default_rng(2)
    E = 6
    for node in range(50):
        mu = rng.normal(0, 1.5, size=E)
        ls = rng.uniform(-3, 1, size=E)
        z = oracle.gaussian_head(np.concatenate([mu, ls]), 5, 9, node)
        eps = np.array([oracle.normal(5, 9, node, e) for e in range(E)])
        u = mu + np.exp(ls) * eps
        # compared as shares: 1 + tanh(u) cancels in float64 for large negative u
        np.testing.assert_allclose(np.exp(z), (1.0 + np.tanh(u)) / 2.0, rtol=1e-12, atol=1e-15)


def test_head_clamps_log_sigma():
    mu = np.array([0.3, -0.2])
    eps = np.array([oracle.normal(1, 1, 10, e) for e in range(2)])
    for ls, eff in [(np.array([5.0, 9.0]), 2.0), (np.array([-50.0, -21.0]), -20.0)]:
        z = oracle.gaussian_head(np.concatenate([mu, ls]), 1, 1, 10)
        u = mu + np.exp(eff) * eps
        np.testing.assert_allclose(np.exp(z), (1.0 + np.tanh(u)) / 2.0, rtol=1e-12, atol=1e-15)


def test_head_small_sigma_limit_is_the_mean():
    mu = np.linspace(-4, 4, 9)
    z = oracle.gaussian_head(np.concatenate([mu, np.full(9, -20.0)]), 3, 4, 5)
    np.testing.assert_allclose(z, -np.log1p(np.exp(-2.0 * mu)), rtol=1e-7)


@pytest.mark.parametrize("rounding", ["lr", "hh"])
def test_gaussian_tree_equals_rollouts(rounding):
    cfg = tt.SMALL.with_head("gaussian").with_rounding(rounding)
    w = wl.make_weights(cfg, 23)
    assert w[-1][0].shape == (2 * cfg.num_ue, cfg.hidden[-1])
    ue = wl.make_ue_state(cfg.num_ue, 24)
    actor = oracle.Actor(w)
    alloc, logits, _ = oracle.build_tree(cfg, w, ue, actor=actor, seed=99, tti=1234)
    K, M = cfg.max_arrival, cfg.num_minislots
    for seq in itertools.product(range(K + 1), repeat=M):
        rows = oracle.rollout(cfg, w, ue, seq, actor=actor, seed=99, tti=1234)
        for tau in range(1, M + 1):
            node = oracle.node_index(K, seq[:tau])
            assert alloc[node].tolist() == rows[tau - 1].tolist(), (seq, tau)
    parity.check_invariants(cfg, ue, alloc)
    again, logits2, _ = oracle.build_tree(cfg, w, ue, actor=actor, seed=99, tti=1234)
    assert np.array_equal(again, alloc) and np.array_equal(logits2, logits)
    other, logits3, _ = oracle.build_tree(cfg, w, ue, actor=actor, seed=99, tti=1235)
    assert not np.array_equal(logits3, logits)
    # logits are log-shares: every evaluated node's are negative
    K1 = K + 1
    evaluated = [oracle.level_offset(K, tau) + i for tau in range(1, M + 1) for i in range(K1 ** tau) if i % K1]
    assert (logits[evaluated] < 0).all()


def test_conditioned_gaussian_uses_node_counters():
    cfg = tt.SMALL.with_head("gaussian")
    w = wl.make_weights(cfg, 25)
    ue = wl.make_ue_state(cfg.num_ue, 26)
    alloc, logits, _ = oracle.build_tree(cfg, w, ue, seed=3, tti=4)
    a2, z2, _ = oracle.eval_conditioned(cfg, w, ue, alloc, seed=3, tti=4)
    assert np.array_equal(a2, alloc.astype(np.int32)) and np.allclose(z2, logits, rtol=0, atol=0)
