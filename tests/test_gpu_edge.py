"""GPU parity on the method's degenerate cases, with hand-set actor weights,
through the C ABI, at the E = 8, K = 3, M = 7 tree (34 -> 256 -> 256 -> 8).

Every layer's weight matrix is zero, so each node's logits are the output
bias whatever its state:
- equal output biases: a uniform softmax, so the shares of all uncapped UEs
  are exactly equal and the largest-remainder cut falls between exact ties,
  which go to the lower UE index (a reading of Eq. (7)'s rounding step);
- output bias ln R_e (the paper's RP benchmark policy, Sec. VII): shares in
  proportion to the scheduled RBs, landing on integers and on caps, with exact
  ties between UEs of equal R_e;
- UE states whose total capacity sum R is at or below the demand U k, where
  the allocation is R itself (T = min(U k, sum R)).

Exact ties are decided identically on both sides (the same inputs give the
same floating-point values in every lane), so these cases demand a bit-exact
codebook, boundary cases included, in FP32 and BF16, on both kernel paths.
"""
import numpy as np
import pytest

import oracle
from paper_2506_00167_amd import cyrus
from paper_2506_00167_amd import workload as wl
from tests import parity

pytestmark = pytest.mark.gpu

C2 = wl.TREE_E8K3


def zero_actor(cfg, out_bias, hidden_bias=0.125):
    """Zero weight matrices; hidden biases constant, output bias as given."""
    dims = cfg.dims
    layers = []
    for l in range(len(dims) - 1):
        w = np.zeros((dims[l + 1], dims[l]), np.float32)
        last = l == len(dims) - 2
        b = np.asarray(out_bias, np.float32) if last else np.full(dims[l + 1], hidden_bias, np.float32)
        layers.append((w, b))
    return layers


def rp_bias(ue):
    """Logits ln R_e: softmax shares R_e / sum R (UEs with R_e = 0 get a
    logit far below the others; their cap of zero decides them anyway)."""
    rb = np.asarray(ue.rb, np.float64)
    return np.where(rb > 0, np.log(np.maximum(rb, 1.0)), -60.0).astype(np.float32)


def fixed_state(rb, seed=5):
    base = wl.make_ue_state(len(rb), seed)
    return wl.UEState(rb=np.asarray(rb, np.int32), mcs=base.mcs, sinr_db=base.sinr_db)


STATES = {
    "random": lambda: wl.make_ue_state(C2.num_ue, wl.ue_seed(0)),
    "edge": lambda: wl.make_ue_state_edge(C2.num_ue, wl.ue_seed(3)),
    "equal-rb": lambda: fixed_state([12] * 8),
    # equal RB counts whose remainders meet at the largest-remainder cut
    # (demand 2 and 4 RBs; and 4 and 6 RBs)
    "pairs": lambda: fixed_state([31, 23, 16, 32, 23, 31, 8, 19]),
    "triples": lambda: fixed_state([27, 14, 14, 14, 13, 30, 13, 13]),
    "over-capacity": lambda: fixed_state([1, 0, 1, 0, 0, 1, 0, 0]),
    "at-capacity": lambda: fixed_state([2, 0, 0, 1, 0, 0, 0, 3]),
    "unscheduled": lambda: fixed_state([0] * 8),
}


def _run(cfg, weights, ue, force_level):
    cb = cyrus.Codebook(cfg, weights, export_logits=True, force_level=force_level)
    print(f"[edge] {cfg.precision} path={cb.kernel_path} rb={list(np.asarray(ue.rb))}", flush=True)
    cb.build(ue)
    cb.wait()
    alloc, logits = cb.export()
    cb.close()
    return alloc, logits


def _check_exact(cfg, weights, ue, alloc, logits, out_bias, tag):
    parity.check_invariants(cfg, ue, alloc)
    prec = "exact" if cfg.precision == "fp32" else cfg.precision
    rep = parity.compare(cfg, weights, ue, alloc, logits, precision=prec, logit_tol=0.0)
    print(f"[edge] {tag}: {rep.as_dict()}", flush=True)
    assert rep.cond_mismatch == 0, f"{tag}: {rep.cond_mismatch} conditioned disagreements"
    assert rep.free_mismatch == 0, f"{tag}: {rep.free_mismatch} free-running disagreements"
    # the exported logits are the output bias itself at every evaluated node
    K = cfg.max_arrival
    for tau in range(1, cfg.num_minislots + 1):
        off = oracle.level_offset(K, tau)
        width = (K + 1) ** tau
        ev = off + np.nonzero(np.arange(width) % (K + 1))[0]
        assert np.array_equal(logits[ev], np.broadcast_to(np.asarray(out_bias, np.float32), (ev.size, cfg.num_ue)))


def _ties(cfg, weights, ue, alloc, precision):
    """Evaluated nodes whose largest-remainder cut falls between equal
    remainders (oracle margin exactly zero)."""
    _, _, marg = oracle.eval_conditioned(cfg, weights, ue, alloc, precision=precision)
    K = cfg.max_arrival
    n = np.arange(cfg.num_nodes)
    evals = np.array([parity.level_of(cfg, int(i)) > 0 for i in n]) & (
        np.array([(int(i) - oracle.level_offset(K, parity.level_of(cfg, int(i)))) % (K + 1) for i in n]) != 0)
    return int(np.count_nonzero(marg[evals] == 0.0))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("force_level", [False, True])
@pytest.mark.parametrize("state", ["random", "edge", "over-capacity", "unscheduled"])
def test_uniform_logits_ties_to_lower_index(precision, force_level, state):
    cfg = C2.with_precision(precision)
    out_bias = np.full(cfg.num_ue, 0.25, np.float32)
    weights = zero_actor(cfg, out_bias)
    ue = STATES[state]()
    alloc, logits = _run(cfg, weights, ue, force_level)
    tag = f"uniform {precision} level={force_level} {state}"
    _check_exact(cfg, weights, ue, alloc, logits, out_bias, tag)
    if state == "random":
        # E = 8 equal shares of T in {2, 4, 6}: every evaluated node's cut
        # falls between exact ties, and the lower indices win
        assert _ties(cfg, weights, ue, alloc, "exact" if precision == "fp32" else precision) == cfg.num_evals
        lvl1 = alloc[1:1 + cfg.max_arrival + 1]
        assert lvl1[1].tolist() == [1, 1, 0, 0, 0, 0, 0, 0]
        assert lvl1[2].tolist() == [1, 1, 1, 1, 0, 0, 0, 0]
        assert lvl1[3].tolist() == [1, 1, 1, 1, 1, 1, 0, 0]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("force_level", [False, True])
@pytest.mark.parametrize("state", ["random", "equal-rb", "pairs", "triples", "at-capacity"])
def test_rp_actor(precision, force_level, state):
    cfg = C2.with_precision(precision)
    ue = STATES[state]()
    out_bias = rp_bias(ue)
    weights = zero_actor(cfg, out_bias)
    alloc, logits = _run(cfg, weights, ue, force_level)
    tag = f"rp {precision} level={force_level} {state}"
    _check_exact(cfg, weights, ue, alloc, logits, out_bias, tag)
    if state in ("equal-rb", "pairs", "triples"):
        assert _ties(cfg, weights, ue, alloc, "exact" if precision == "fp32" else precision) > 0
    if state == "at-capacity":
        # sum R = 6 = U K: the k = 3 children puncture exactly R at every level
        R = np.asarray(ue.rb)
        K = cfg.max_arrival
        for tau in range(1, cfg.num_minislots + 1):
            off = oracle.level_offset(K, tau)
            full = alloc[off + np.arange(K, (K + 1) ** tau, K + 1)]
            assert (full == R[None, :]).all()
