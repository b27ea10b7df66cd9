"""Parity of the HIP codebook builder with the FP64 oracle, through the C ABI.

FP32: conditioned-mode allocations must match the oracle at every node except
where the oracle's float64 decision margin is below 1e-6 (counted and
reported); free-running disagreements must descend from conditioned ones.
Logits within 1e-4. BF16: against the oracle run in BF16, every disagreement
explained by the node's measured logit error (tests/parity.py).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2506_00167_amd import cyrus
from paper_2506_00167_amd import workload as wl
from tests import parity

pytestmark = pytest.mark.gpu

FP32_LOGIT_TOL = 1e-4

# Subtree-kernel shapes at the edges of the first layer's per-node inputs
# (c, tau, k: E + 2 of them): exactly one 16-wide FP32 chunk at E = 14, two
# chunks at E = 16.
SUBTREE_WIDE = [
    dict(num_ue=14, max_arrival=3, num_minislots=4, hidden=(128, 128)),
    dict(num_ue=16, max_arrival=2, num_minislots=4, hidden=(256, 256)),
]

# Subtree-kernel shapes whose levels hold more rows than one pass (48 rows in
# FP32, 64 in BF16/FP8), or a partly filled pass: K = 7, M = 5 has subtree
# levels of 7, 56 and 448 rows (FP32: nine full passes and a 16-row tail);
# K = 4, M = 6 has 100 rows (FP32: 48 + 48 + a 4-row tail on the vector ALU);
# K = 5, M = 5 has a 30-row level (two of the pass's 16-row tiles live).
SUBTREE_MULTIPASS = [
    dict(num_ue=8, max_arrival=7, num_minislots=5, hidden=(256, 256)),
    dict(num_ue=16, max_arrival=4, num_minislots=6, hidden=(128, 128)),
    dict(num_ue=8, max_arrival=5, num_minislots=5, hidden=(256, 256)),
]

# The largest tree and actor the configuration accepts: E = 32, K = 7, M = 7,
# U = 5 (M K U = 245; the carried state is 8-bit), four 512-wide hidden
# layers. 2,396,745 nodes, 2,097,151 evaluations.
MAX_TREE = dict(num_ue=32, max_arrival=7, num_minislots=7, rb_per_unit=5, hidden=(512, 512, 512, 512))


def _build(cfg, weights, ue, **kw):
    cb = cyrus.Codebook(cfg, weights, export_logits=True, **kw)
    print(f"[build] {cfg} path={cb.kernel_path}", flush=True)
    cb.build(ue)
    cb.wait()
    alloc, logits = cb.export()
    return cb, alloc, logits


def _report(tag, rep, exact=True):
    rep.check(tag, exact)


@pytest.mark.parametrize("force_level", [True, False])
@pytest.mark.parametrize("edge", [False, True])
def test_tiny_fp32(force_level, edge):
    cfg = wl.TINY
    weights = wl.make_weights(cfg, wl.WEIGHT_SEEDS["tiny-e4k2"])
    ue = (wl.make_ue_state_edge if edge else wl.make_ue_state)(cfg.num_ue, wl.ue_seed(1))
    cb, alloc, logits = _build(cfg, weights, ue, force_level=force_level)
    parity.check_invariants(cfg, ue, alloc)
    rep = parity.compare(cfg, weights, ue, alloc, logits, logit_tol=FP32_LOGIT_TOL)
    _report(f"tiny level={force_level} edge={edge}", rep)
    cb.close()


@pytest.mark.parametrize("force_level", [True, False])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tree_e8k3_fp32(force_level, seed):
    cfg = wl.TREE_E8K3
    weights = wl.make_weights(cfg, wl.WEIGHT_SEEDS["tree-e8k3"])
    ue = wl.make_ue_state(cfg.num_ue, wl.ue_seed(seed))
    cb, alloc, logits = _build(cfg, weights, ue, force_level=force_level)
    parity.check_invariants(cfg, ue, alloc)
    rep = parity.compare(cfg, weights, ue, alloc, logits, logit_tol=FP32_LOGIT_TOL)
    _report(f"e8k3 level={force_level} seed={seed}", rep)
    cb.close()


@pytest.mark.parametrize("shape", [
    dict(num_ue=1, max_arrival=1, num_minislots=7, hidden=(128,)),
    dict(num_ue=10, max_arrival=2, num_minislots=1, hidden=(128,)),            # the paper's depth-1 codebook
    dict(num_ue=16, max_arrival=4, num_minislots=3, hidden=(512, 512)),
    dict(num_ue=32, max_arrival=2, num_minislots=4, hidden=(256, 384, 128)),  # 32 UEs: two output tiles
    dict(num_ue=5, max_arrival=7, num_minislots=2, rb_per_unit=3, hidden=(256, 256, 256, 256)),
    *SUBTREE_WIDE,
    *SUBTREE_MULTIPASS,
])
def test_shapes_fp32(shape):
    cfg = wl.TreeConfig(**shape)
    weights = wl.make_weights(cfg, 31)
    ue = wl.make_ue_state(cfg.num_ue, 32)
    for force_level in (True, False):
        cb, alloc, logits = _build(cfg, weights, ue, force_level=force_level)
        parity.check_invariants(cfg, ue, alloc)
        rep = parity.compare(cfg, weights, ue, alloc, logits, logit_tol=FP32_LOGIT_TOL)
        _report(f"{shape} level={force_level}", rep)
        cb.close()


def test_latency_path_is_selected():
    wide = [wl.TreeConfig(**s) for s in SUBTREE_WIDE + SUBTREE_MULTIPASS]
    for cfg in (wl.TINY, wl.TREE_E8K3, wl.PAPER_DEPTH1, wl.TREE_E8K3.with_precision("bf16"), *wide):
        cb = cyrus.Codebook(cfg, wl.make_weights(cfg, 1), act_scale=None)
        assert cb.kernel_path == "subtree", cfg
        cb.close()
    cb = cyrus.Codebook(wl.TREE_E8K3, wl.make_weights(wl.TREE_E8K3, 1), force_level=True)
    assert cb.kernel_path == "level"
    cb.close()


def test_subtree_bf16_wide():
    cfg = wl.TreeConfig(precision="bf16", **SUBTREE_WIDE[1])
    weights = wl.make_weights(cfg, 33)
    ue = wl.make_ue_state(cfg.num_ue, 34)
    cb, alloc, logits = _build(cfg, weights, ue)
    assert cb.kernel_path == "subtree"
    parity.check_invariants(cfg, ue, alloc)
    rep = parity.compare(cfg, weights, ue, alloc, logits, precision="bf16", logit_tol=2e-3)
    _report("bf16 e16k2 subtree", rep, exact=False)
    cb.close()


@pytest.mark.parametrize("shape", [SUBTREE_MULTIPASS[0], SUBTREE_MULTIPASS[2]])
def test_subtree_bf16_multipass(shape):
    cfg = wl.TreeConfig(precision="bf16", **shape)
    weights = wl.make_weights(cfg, 35)
    ue = wl.make_ue_state(cfg.num_ue, 36)
    cb, alloc, logits = _build(cfg, weights, ue)
    assert cb.kernel_path == "subtree"
    parity.check_invariants(cfg, ue, alloc)
    rep = parity.compare(cfg, weights, ue, alloc, logits, precision="bf16", logit_tol=2e-3)
    _report(f"bf16 {shape} subtree", rep, exact=False)
    cb.close()


@pytest.mark.parametrize("prec,tol", [("fp32", FP32_LOGIT_TOL), ("bf16", 2e-3)])
def test_maximum_tree_sampled(prec, tol):
    """Every node against the invariants; a sample of nodes, with the path
    of all-K arrivals, recomputed by the oracle from the GPU's parent states."""
    cfg = wl.TreeConfig(precision=prec, **MAX_TREE)
    weights = wl.make_weights(cfg, 41)
    ue = wl.make_ue_state(cfg.num_ue, wl.ue_seed(41))
    cb, alloc, logits = _build(cfg, weights, ue)
    assert cb.kernel_path == "level"
    parity.check_invariants(cfg, ue, alloc)
    last = cfg.num_nodes - 1
    nodes = np.union1d(wl.sample_nodes(cfg, 400, seed=43), [last, *parity.ancestors(cfg, last)])
    rep = parity.compare(cfg, weights, ue, alloc, logits, nodes=nodes,
                         precision="exact" if prec == "fp32" else prec, logit_tol=tol)
    _report(f"{prec} maximum tree sampled", rep, exact=prec == "fp32")
    cb.close()


def test_lookup_matches_export_and_oracle_rollouts():
    cfg = wl.TREE_E8K3
    weights = wl.make_weights(cfg, wl.WEIGHT_SEEDS["tree-e8k3"])
    ue = wl.make_ue_state(cfg.num_ue, wl.ue_seed(3))
    cb, alloc, _ = _build(cfg, weights, ue)
    seqs = wl.random_sequences(cfg, 200, seed=5)
    for seq in seqs:
        for tau in range(1, cfg.num_minislots + 1):
            row = cb.lookup(seq[:tau])
            assert row.tolist() == alloc[oracle.node_index(cfg.max_arrival, seq[:tau])].tolist()
    cb.close()


def test_deterministic_and_device_build_equal():
    import torch
    cfg = wl.TREE_E8K3
    weights = wl.make_weights(cfg, wl.WEIGHT_SEEDS["tree-e8k3"])
    ue = wl.make_ue_state(cfg.num_ue, wl.ue_seed(4))
    for force_level in (True, False):
        cb = cyrus.Codebook(cfg, weights, export_logits=True, force_level=force_level)
        cb.build(ue)
        a1, l1 = cb.export()
        cb.build(ue)
        a2, l2 = cb.export()
        cb.build_device(cyrus.ue_device_tensor(ue))
        torch.cuda.synchronize()
        a3, l3 = cb.export()
        assert np.array_equal(a1, a2) and np.array_equal(l1, l2)
        assert np.array_equal(a1, a3) and np.array_equal(l1, l3)
        cb.close()


def test_batch_equals_single_builds():
    import torch
    cfgs = [wl.TINY, wl.TREE_E8K3, wl.TreeConfig(num_ue=6, max_arrival=2, num_minislots=5, hidden=(256, 256))]
    cbs, ues, refs = [], [], []
    for i, cfg in enumerate(cfgs):
        weights = wl.make_weights(cfg, 40 + i)
        ue = wl.make_ue_state(cfg.num_ue, 50 + i)
        single = cyrus.Codebook(cfg, weights, export_logits=True, force_level=True)
        single.build(ue)
        refs.append(single.export())
        single.close()
        cbs.append(cyrus.Codebook(cfg, weights, export_logits=True, force_level=True))
        ues.append(cyrus.ue_device_tensor(ue))
    cyrus.build_batch_device(cbs, ues)
    torch.cuda.synchronize()
    for cb, (ra, rl) in zip(cbs, refs):
        a, l = cb.export()
        assert np.array_equal(a, ra) and np.array_equal(l, rl)
        cb.close()


def test_set_weights_equals_fresh_codebook():
    cfg = wl.TINY
    w1 = wl.make_weights(cfg, 61)
    w2 = wl.make_weights(cfg, 62)
    ue = wl.make_ue_state(cfg.num_ue, 63)
    cb = cyrus.Codebook(cfg, w1, export_logits=True)
    cb.build(ue)
    first, _ = cb.export()
    cb.set_weights(w2)
    cb.build(ue)
    a, l = cb.export()
    fresh = cyrus.Codebook(cfg, w2, export_logits=True)
    fresh.build(ue)
    fa, fl = fresh.export()
    assert np.array_equal(a, fa) and np.array_equal(l, fl)
    assert not np.array_equal(first, a)
    cb.close()
    fresh.close()


def test_errors_do_not_enqueue():
    cfg = wl.TINY
    weights = wl.make_weights(cfg, 1)
    cb = cyrus.Codebook(cfg, weights)
    with pytest.raises(cyrus.CyrusError) as ei:
        cb.lookup([1])
    assert ei.value.status == -5  # lookup before any build
    bad = wl.make_ue_state(cfg.num_ue, 1)
    bad.rb[0] = 300
    with pytest.raises(cyrus.CyrusError) as ei:
        cb.build(bad)
    assert ei.value.status == -2
    cb.build(wl.make_ue_state(cfg.num_ue, 2))
    with pytest.raises(cyrus.CyrusError):
        cb.lookup([3])  # arrival above K
    with pytest.raises(cyrus.CyrusError):
        cb.lookup([1] * 8)  # deeper than M
    cb.close()


def test_oru_assemble_matches_oracle():
    cfg = wl.TREE_E8K3
    weights = wl.make_weights(cfg, wl.WEIGHT_SEEDS["tree-e8k3"])
    ue = wl.make_ue_state(cfg.num_ue, wl.ue_seed(5))
    cb, alloc, _ = _build(cfg, weights, ue)
    rng = np.random.default_rng(10)
    for _ in range(100):
        # URLLC arrivals per mini-slot: 12 URLLC UEs, each with a packet w.p. 0.08
        raw = rng.binomial(12, 0.08, size=cfg.num_minislots) * int(rng.integers(1, 4))
        c_in = int(rng.integers(0, 3))
        served, y, carry = cb.assemble(raw, c_in)
        o_served, _, o_carry = oracle.oru_assemble(cfg, weights, ue, raw, c_in)
        assert served.tolist() == o_served.tolist() and carry == o_carry
        for tau in range(1, cfg.num_minislots + 1):
            node = oracle.node_index(cfg.max_arrival, served[:tau])
            assert y[tau - 1].tolist() == alloc[node].tolist()
    cb.close()


def _skewed(weights, E, seed):
    """Uneven output biases, so that shares are uneven and the two roundings
    part ways at many nodes."""
    rng = np.random.default_rng(seed)
    w = list(weights)
    w[-1] = (w[-1][0], rng.uniform(-3.0, 3.0, size=E).astype(np.float32))
    return w


@pytest.mark.parametrize("shape", [
    dict(num_ue=8, max_arrival=3, rb_per_unit=5, hidden=(256, 256)),
    dict(num_ue=4, max_arrival=2, rb_per_unit=9, hidden=(256, 256)),
    dict(num_ue=24, max_arrival=2, num_minislots=4, rb_per_unit=6, hidden=(256, 128)),  # 32-lane groups
    dict(num_ue=8, max_arrival=4, num_minislots=6, rb_per_unit=5, hidden=(128, 128)),    # 100-row levels
])
@pytest.mark.parametrize("force_level", [True, False])
def test_huntington_hill_fp32(shape, force_level):
    cfg = wl.TreeConfig(rounding="hh", **shape)
    weights = _skewed(wl.make_weights(cfg, 41), cfg.num_ue, 42)
    ue = wl.make_ue_state(cfg.num_ue, 43)
    cb, alloc, logits = _build(cfg, weights, ue, force_level=force_level)
    parity.check_invariants(cfg, ue, alloc)
    rep = parity.compare(cfg, weights, ue, alloc, logits, logit_tol=FP32_LOGIT_TOL)
    _report(f"hh {shape} level={force_level} path={cb.kernel_path}", rep)
    # the flag reaches the kernels: largest remainder gives another codebook
    cb_lr, alloc_lr, _ = _build(cfg.with_rounding("lr"), weights, ue, force_level=force_level)
    assert not np.array_equal(alloc, alloc_lr)
    cb_lr.close()
    cb.close()


@pytest.mark.parametrize("shape", [
    dict(num_ue=8, max_arrival=3, rb_per_unit=3, hidden=(256, 256)),
    dict(num_ue=4, max_arrival=2, rb_per_unit=5, hidden=(128,)),
    dict(num_ue=16, max_arrival=4, num_minislots=3, hidden=(256, 256)),   # 2E = 32: two output tiles
    dict(num_ue=8, max_arrival=4, num_minislots=6, rb_per_unit=3, hidden=(128, 128)),  # 100-row levels
    # the paper's own shape (Sec. VII): depth 1, E = 10, two arrival branches,
    # one hidden layer of 128; 2E = 20 outputs take the level path
    dict(num_ue=10, max_arrival=2, num_minislots=1, hidden=(128,)),
])
@pytest.mark.parametrize("rounding", ["lr", "hh"])
def test_gaussian_head_fp32(shape, rounding):
    cfg = wl.TreeConfig(head="gaussian", rounding=rounding, **shape)
    weights = wl.make_weights(cfg, 51)
    ue = wl.make_ue_state(cfg.num_ue, 52)
    seed, tti = 0x1234_5678_9ABC, 77_000_001
    for force_level in (True, False):
        cb = cyrus.Codebook(cfg, weights, export_logits=True, force_level=force_level)
        cb.set_rng(seed, tti)
        print(f"[build] gaussian {shape} {rounding} level={force_level} path={cb.kernel_path}", flush=True)
        cb.build(ue)
        cb.wait()
        alloc, logits = cb.export()
        parity.check_invariants(cfg, ue, alloc)
        rep = parity.compare(cfg, weights, ue, alloc, logits, logit_tol=FP32_LOGIT_TOL, seed=seed, tti=tti)
        _report(f"gaussian {shape} {rounding} level={force_level} path={cb.kernel_path}", rep)
        # the same key and TTI repeat the codebook; the next TTI draws anew
        cb.build(ue)
        cb.wait()
        again, logits2 = cb.export()
        assert np.array_equal(again, alloc) and np.array_equal(logits2, logits)
        cb.set_rng(seed, tti + 1)
        cb.build(ue)
        cb.wait()
        assert not np.array_equal(cb.export()[1], logits)
        cb.close()


def test_gaussian_head_bf16_and_batch():
    import torch
    cfg = wl.TreeConfig(num_ue=8, max_arrival=3, hidden=(256, 256), precision="bf16", head="gaussian")
    weights = wl.make_weights(cfg, 53)
    ues = [wl.make_ue_state(cfg.num_ue, 54 + j) for j in range(3)]
    cells = []
    for j in range(3):
        c = cyrus.Codebook(cfg, weights, export_logits=True, force_level=True)
        c.set_rng(99, 1000 + j)
        cells.append(c)
    dev = [cyrus.ue_device_tensor(u) for u in ues]
    cyrus.build_batch_device(cells, dev)
    torch.cuda.synchronize()
    for j, c in enumerate(cells):
        alloc, logits = c.export()
        # A hidden activation that the FP32 and FP64 sums place on either side
        # of a BF16 rounding boundary differs by one BF16 unit (2^-8 relative);
        # the head multiplies an error in log sigma by up to 2 sigma |eps|
        # (sigma <= e^2), so the same-precision logit bound of 2e-3 for
        # softmax logits becomes 2e-2 here.
        rep = parity.compare(cfg, weights, ues[j], alloc, logits, precision="bf16", logit_tol=2e-2, seed=99,
                             tti=1000 + j)
        _report(f"gaussian bf16 batch cell {j}", rep, exact=False)
        c.build(ues[j])
        c.wait()
        assert np.array_equal(c.export()[0], alloc)
        c.close()


def test_refresh_waits_for_builds_in_flight():
    """Two weight refreshes while builds run on another stream: the second
    one overwrites the buffer those builds read, so it must wait for them.
    The last build before the refreshes gives the old weights' codebook; the
    next one gives the new weights' codebook."""
    import torch
    cfg = wl.TREE_E8K3
    w1, w2, w3 = (wl.make_weights(cfg, s) for s in (41, 42, 43))
    ue = wl.make_ue_state(cfg.num_ue, wl.ue_seed(4))

    def reference(w):
        r = cyrus.Codebook(cfg, w)
        r.build(ue)
        a, _ = r.export()
        r.close()
        return a

    ref1, ref3 = reference(w1), reference(w3)
    s_build, s_refresh = torch.cuda.Stream(), torch.cuda.Stream()
    cb = cyrus.Codebook(cfg, w1, stream=s_build)
    ue_dev = cyrus.ue_device_tensor(ue)
    torch.cuda.synchronize()
    for _ in range(300):  # about 14 ms of builds in flight on s_build
        cb.build_device(ue_dev)
    v2, v3 = cyrus._WeightsView(w2), cyrus._WeightsView(w3)
    cyrus.cyrus_codebook_set_weights(cb.handle, v2.struct, s_refresh)
    cyrus.cyrus_codebook_set_weights(cb.handle, v3.struct, s_refresh)
    cb.wait()
    old, _ = cb.export()
    assert np.array_equal(old, ref1), "a build enqueued before the refresh saw the new weights"
    cb.build(ue)
    new, _ = cb.export()
    assert np.array_equal(new, ref3)
    cb.close()


def test_build_batch_host_states():
    """The host-state batch: UE states staged by the call, codebooks in each
    handle's pinned mirror afterwards, equal to single builds."""
    cfgs = [wl.TINY, wl.TreeConfig(num_ue=6, max_arrival=2, num_minislots=6, hidden=(256, 256)), wl.TINY]
    cbs = [cyrus.Codebook(c, wl.make_weights(c, 50 + i), force_level=True) for i, c in enumerate(cfgs)]
    ues = [wl.make_ue_state(c.num_ue, 60 + i) for i, c in enumerate(cfgs)]
    cyrus.build_batch(cbs, ues)
    for cb, ue in zip(cbs, ues):
        cb.wait()
        batch, _ = cb.export()
        assert cb.lookup([0]).tolist() == [0] * cb.cfg.num_ue
        cb.build(ue)
        single, _ = cb.export()
        assert np.array_equal(batch, single)
        parity.check_invariants(cb.cfg, ue, batch)
        cb.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_hidden_widths_padded(precision):
    """Hidden widths that are multiples of 32 but not of 128 (zero-padded to
    128 inside the library) against the oracle's exact widths."""
    cfg = wl.TreeConfig(num_ue=6, max_arrival=3, num_minislots=5, hidden=(160, 96), precision=precision)
    weights = wl.make_weights(cfg, 71)
    ue = wl.make_ue_state(cfg.num_ue, 72)
    for force_level in (True, False):
        cb, alloc, logits = _build(cfg, weights, ue, force_level=force_level)
        parity.check_invariants(cfg, ue, alloc)
        if precision == "fp32":
            rep = parity.compare(cfg, weights, ue, alloc, logits, logit_tol=FP32_LOGIT_TOL)
            _report(f"hidden 160/96 level={force_level}", rep)
        else:
            rep = parity.compare(cfg, weights, ue, alloc, logits, precision="bf16", logit_tol=2e-3)
            _report(f"bf16 hidden 160/96 level={force_level}", rep, exact=False)
        cb.close()


def test_fp8_scale_outside_block_scale_range_is_refused():
    """Each FP8 layer's combined output scale (weight scale x its input scale
    / the next layer's input scale) is applied as an E8M0 block scale, which
    holds 2^-126..2^127: act_scale values that push it outside are refused
    at creation and at a weight refresh, and the old weights stay usable."""
    cfg = wl.TREE_E8K3.with_precision("fp8")
    weights = wl.make_weights(cfg, wl.WEIGHT_SEEDS["tree-e8k3"])
    bad = [2.0 ** -100, 2.0 ** 100, 1.0]
    with pytest.raises(cyrus.CyrusError) as ei:
        cyrus.Codebook(cfg, weights, act_scale=bad)
    assert ei.value.status == -2
    good = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fp8_act_scales.json")))[
        f"tree-e8k3/{wl.WEIGHT_SEEDS['tree-e8k3']}"]
    cb = cyrus.Codebook(cfg, weights, act_scale=good)
    ue = wl.make_ue_state(cfg.num_ue, wl.ue_seed(0))
    cb.build(ue)
    cb.wait()
    first = cb.export()[0]
    with pytest.raises(cyrus.CyrusError) as ei:
        cb.set_weights(weights, act_scale=bad)
    assert ei.value.status == -2
    cb.build(ue)
    cb.wait()
    assert np.array_equal(cb.export()[0], first)
    cb.close()
