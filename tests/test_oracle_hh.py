"""Pins of the oracle's Huntington-Hill rounding (the paper's rounding step,
Sec. IV-B, citing Balinski and Young), independent of its own code:

- the divisor form: a Huntington-Hill allocation is min(R_e, r(x_e / d)) for
  some divisor d, where r rounds y up exactly when y is at least the geometric
  mean sqrt(n (n+1)) of its neighbouring integers (so every positive y < 1
  rounds up to 1). The oracle computes the priority form; the test scans
  divisors instead, which is a different computation of the same definition;
- hand-worked cases, chosen where Huntington-Hill and largest remainder differ;
- house monotonicity and scale invariance, which every divisor method has;
- the margin: moving the shares by less than it never changes the result.
"""
import dataclasses
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2506_00167_amd import workload as wl
from tests import parity
from tests import test_oracle_tree as tt


def _gm_round(y: float) -> int:
    if y <= 0.0:
        return 0
    f = math.floor(y)
    return f + 1 if y >= math.sqrt(f * (f + 1)) else f


def _divisor_allocation(x, R, T):
    """Scan the critical divisors x_e / sqrt(n (n+1)) and their neighbours for
    one whose capped geometric-mean rounding sums to T."""
    crit = set()
    for xe, re in zip(x, R):
        if xe <= 0:
            continue
        for n in range(1, int(re) + 2):
            crit.add(xe / math.sqrt(n * (n + 1)))
    cands = sorted(crit)
    probes = []
    for i, c in enumerate(cands):
        probes += [c * (1 - 1e-9), c * (1 + 1e-9)]
        if i + 1 < len(cands):
            probes.append(0.5 * (c + cands[i + 1]))
    probes += [1.0, (cands[-1] * 2 if cands else 1.0), (cands[0] / 2 if cands else 1.0)]
    sols = []
    for d in probes:
        a = [min(int(re), _gm_round(xe / d)) for xe, re in zip(x, R)]
        if sum(a) == T:
            sols.append(tuple(a))
    return sols


def _quotas(rng, E, T, R):
    p = rng.dirichlet(np.ones(E) * 0.7)
    x, _ = oracle.capped_scale(p, R, T)
    return x


def test_matches_divisor_form_random():
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(400):
        E = int(rng.integers(2, 6))
        R = rng.integers(1, 9, size=E).astype(np.int32)
        T = int(rng.integers(1, R.sum() + 1))
        x = _quotas(rng, E, T, R)
        if T < int((x > 0).sum()):
            continue  # no Huntington-Hill allocation exists (checked below)
        a = oracle.huntington_hill(x, R, T)
        sols = _divisor_allocation(x, R, T)
        assert sols, (x, R, T)
        assert tuple(int(v) for v in a) in sols, (x, R, T, a, sols)
        checked += 1
    assert checked > 200


def test_hand_case_differs_from_largest_remainder():
    # shares 0.3, 0.3, 4.4 of T = 5: largest remainder gives [0, 0, 5]; every
    # positive share is owed a unit under Huntington-Hill, then the third UE
    # takes the next two (4.4/sqrt(2) = 3.11, then 4.4/sqrt(6) = 1.80)
    x = np.array([0.3, 0.3, 4.4])
    R = np.array([8, 8, 8], dtype=np.int32)
    assert oracle.largest_remainder(x, R, 5).tolist() == [0, 0, 5]
    assert oracle.huntington_hill(x, R, 5).tolist() == [1, 1, 3]


def test_hand_case_cap_and_ties():
    # UE 0 is capped at 1; UEs 1 and 2 tie at every step and the tie goes to
    # the lower index: [1,1,1] -> [1,2,1] (2.5/sqrt 2 tie) -> [1,2,2] -> [1,3,2]
    x = np.array([1.0, 2.5, 2.5])
    R = np.array([1, 8, 8], dtype=np.int32)
    assert oracle.huntington_hill(x, R, 6).tolist() == [1, 3, 2]
    assert oracle.huntington_hill(x, R, 5).tolist() == [1, 2, 2]


def test_tie_goes_to_larger_share_then_lower_index():
    # first units (all infinite) with T below the number of positive shares:
    # the largest shares win, equal shares go to the lower index
    assert oracle.huntington_hill([0.2, 0.5, 0.3], [4, 4, 4], 2).tolist() == [0, 1, 1]
    assert oracle.huntington_hill([0.5, 0.3, 0.2], [4, 4, 4], 1).tolist() == [1, 0, 0]
    assert oracle.huntington_hill([0.25, 0.5, 0.25], [4, 4, 4], 2).tolist() == [1, 1, 0]


def test_zero_share_and_cap_never_receive():
    x = np.array([0.0, 3.0, 1.0])
    R = np.array([5, 2, 5], dtype=np.int32)
    a = oracle.huntington_hill(x, R, 4)
    assert a.tolist() == [0, 2, 2]


def test_house_monotone_and_scale_invariant():
    rng = np.random.default_rng(5)
    for _ in range(50):
        E = int(rng.integers(2, 7))
        p = rng.dirichlet(np.ones(E))
        R = np.full(E, 64, dtype=np.int32)
        prev = np.zeros(E, dtype=np.int32)
        for T in range(1, 40):
            a = oracle.huntington_hill(p * T, R, T)
            assert a.sum() == T
            d = a - prev
            assert d.min() >= 0 and d.sum() == 1, (p, T, prev, a)  # one more unit, nobody loses
            assert oracle.huntington_hill(p * 7.25, R, T).tolist() == a.tolist()
            prev = a


def _hh_moves(x, R, T, a, step):
    """Every move of two shares toward each other by `step` (one down, one
    up, kept in [0, R]): returns how many change the Huntington-Hill result."""
    flips = 0
    for i in range(x.size):
        for j in range(x.size):
            if i == j:
                continue
            xp = x.copy()
            xp[i] = max(xp[i] - step, 0.0)
            xp[j] = min(xp[j] + step, float(R[j]))
            flips += oracle.huntington_hill(xp, R, T).tolist() != a.tolist()
    return flips


def test_margin_is_a_safe_distance():
    """No move of the shares by less than the margin in every component
    changes the result (random moves and every two-share move), and some
    two-share move by slightly more does."""
    rng = np.random.default_rng(17)
    tested = 0
    for _ in range(300):
        E = int(rng.integers(2, 7))
        R = rng.integers(1, 7, size=E).astype(np.int32)
        T = int(rng.integers(1, R.sum()))
        p = rng.dirichlet(np.ones(E))
        x, _ = oracle.capped_scale(p, R, T)
        a = oracle.huntington_hill(x, R, T)
        m = oracle.margin_hh(x, R, T, a)
        if not np.isfinite(m) or m <= 1e-9:
            continue
        for _ in range(10):
            dx = rng.uniform(-0.9 * m, 0.9 * m, size=E)
            xp = np.minimum(np.maximum(x + dx, 0.0), R)
            xp[x == 0] = 0.0
            assert oracle.huntington_hill(xp, R, T).tolist() == a.tolist(), (x, dx, m)
        assert _hh_moves(x, R, T, a, 0.999 * m) == 0, (x, R, T, m)
        assert _hh_moves(x, R, T, a, 1.001 * m) > 0, (x, R, T, m)
        tested += 1
    assert tested > 100


def test_margin_is_tight_on_a_swap():
    # two second units in competition: moving the shares by slightly more than
    # the margin (in the right direction) flips the decision
    x = np.array([2.0, 1.9])
    R = np.array([8, 8], dtype=np.int32)
    a = oracle.huntington_hill(x, R, 3)
    assert a.tolist() == [2, 1]
    m = oracle.margin_hh(x, R, 3, a)
    assert 0 < m < 0.1
    assert oracle.huntington_hill(x + np.array([-1.01 * m, 1.01 * m]), R, 3).tolist() == [1, 2]


def test_margin_first_units():
    R = np.array([8, 8, 8], dtype=np.int32)
    # fewer units than positive shares: first units go to the larger shares,
    # and the two at the cut swap once each has moved half their difference
    x = np.array([0.9, 0.5, 0.6])
    a = oracle.huntington_hill(x, R, 2)
    assert a.tolist() == [1, 0, 1]
    m = oracle.margin_hh(x, R, 2, a)
    assert m == pytest.approx(0.05, abs=1e-12)
    assert oracle.huntington_hill(x + [0, 1.01 * m, -1.01 * m], R, 2).tolist() == [1, 1, 0]
    # a held first unit is lost only when its share reaches zero
    x = np.array([0.05, 2.95])
    a = oracle.huntington_hill(x, R[:2], 2)
    assert a.tolist() == [1, 1]
    m = oracle.margin_hh(x, R[:2], 2, a)
    assert m == pytest.approx(0.05, abs=1e-12)
    assert oracle.huntington_hill(x + [-0.99 * m, 0.99 * m], R[:2], 2).tolist() == [1, 1]
    assert oracle.huntington_hill(np.array([0.0, 3.0]), R[:2], 2).tolist() == [0, 2]


def test_allocate_hh_invariants():
    rng = np.random.default_rng(3)
    for _ in range(300):
        E = int(rng.integers(1, 9))
        z = rng.normal(0, 3, size=E)
        R = rng.integers(0, 9, size=E).astype(np.int32)
        U, k = int(rng.integers(1, 4)), int(rng.integers(1, 5))
        a, m, x = oracle.allocate(z, R, U, k, rounding="hh")
        T = min(U * k, int(R.sum()))
        assert a.sum() == T and (a >= 0).all() and (a <= R).all()


@pytest.mark.parametrize("edge", [False, True])
def test_tree_hh_equals_brute_force_rollouts(edge):
    # U = 5 RBs per arrival: T reaches 10 over E = 4 UEs, where the two
    # roundings part ways
    cfg = dataclasses.replace(tt.SMALL, rb_per_unit=5, rounding="hh")
    w = wl.make_weights(cfg, 21)
    # a skewed output bias makes uneven shares, where the roundings differ
    w[-1] = (w[-1][0], np.array([0.0, -2.5, -2.5, 2.5], dtype=np.float32))
    ue = (wl.make_ue_state_edge if edge else wl.make_ue_state)(cfg.num_ue, 22)
    actor = oracle.Actor(w)
    alloc, _, _ = oracle.build_tree(cfg, w, ue, actor=actor)
    lr, _, _ = oracle.build_tree(cfg.with_rounding("lr"), w, ue, actor=actor)
    K, M = cfg.max_arrival, cfg.num_minislots
    for seq in itertools.product(range(K + 1), repeat=M):
        rows = oracle.rollout(cfg, w, ue, seq, actor=actor)
        for tau in range(1, M + 1):
            node = oracle.node_index(K, seq[:tau])
            assert alloc[node].tolist() == rows[tau - 1].tolist(), (seq, tau)
    parity.check_invariants(cfg, ue, alloc)
    if not edge:  # (the edge state's tiny caps leave both roundings no choice)
        assert not np.array_equal(alloc, lr)  # the rounding mode reaches the tree
