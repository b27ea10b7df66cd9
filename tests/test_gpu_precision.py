"""BF16 and FP8 (E4M3) variants of the layer GEMMs, FP32 accumulation, softmax
and rounding in FP32.

Gate: parity with the oracle run in the same reduced precision (weights and
every layer input rounded to the format, products and sums exact): logits
within a tolerance derived from FP32 accumulation plus the occasional
activation that rounds to the neighbouring format value, and every
conditioned-mode disagreement explained by the measured logit error.

Report: max logit error and allocation-disagreement rate of each variant
against the exact FP64 oracle, written to precision_report.json in the
directory named by CYRUS_REPORT_DIR (default: reports/ under the repository).
"""
import json
import os

import numpy as np
import pytest

from paper_2506_00167_amd import cyrus
from paper_2506_00167_amd import workload as wl
from tests import parity

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORT_DIR = os.environ.get("CYRUS_REPORT_DIR", os.path.join(ROOT, "reports"))
SCALES = json.load(open(os.path.join(ROOT, "tests", "golden", "fp8_act_scales.json")))

# Logit tolerance against the same-precision oracle: FP32 accumulation error
# is ~1e-6; an activation that lands on the other side of a rounding boundary
# moves one input by one unit in the last place (2^-8 relative for BF16, 2^-3
# for E4M3) and the logits by that times a weight (|w| < 0.15 here).
SAME_PREC_TOL = {"bf16": 2e-3, "fp8": 5e-2}
REPORT = {}


def _codebook(cfg, weights, act, ue, force_level):
    cb = cyrus.Codebook(cfg, weights, act_scale=act, export_logits=True, force_level=force_level)
    cb.build(ue)
    cb.wait()
    a, l = cb.export()
    path = cb.kernel_path
    cb.close()
    return a, l, path


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("force_level", [True, False])
def test_tree_e8k3_reduced_precision(prec, force_level):
    base = wl.TREE_E8K3
    cfg = base.with_precision(prec)
    seed = wl.WEIGHT_SEEDS["tree-e8k3"]
    weights = wl.make_weights(cfg, seed)
    act = SCALES[f"tree-e8k3/{seed}"] if prec == "fp8" else None
    ue = wl.make_ue_state(cfg.num_ue, wl.ue_seed(7))
    alloc, logits, path = _codebook(cfg, weights, act, ue, force_level)
    parity.check_invariants(cfg, ue, alloc)
    same = parity.compare(cfg, weights, ue, alloc, logits, precision=prec, act_scale=act,
                          logit_tol=SAME_PREC_TOL[prec])
    same.check(f"{prec} {path} vs same-precision oracle", exact=False)
    exact = parity.compare(cfg, weights, ue, alloc, logits, precision="exact")
    print(f"[{prec} {path}] vs FP64 oracle: {exact.as_dict()}", flush=True)
    REPORT[f"tree-e8k3/{prec}/{path}"] = {"vs_same_precision_oracle": same.as_dict(),
                                          "vs_fp64_oracle": exact.as_dict()}
    os.makedirs(REPORT_DIR, exist_ok=True)
    with open(os.path.join(REPORT_DIR, "precision_report.json"), "w") as f:
        json.dump(REPORT, f, indent=1)


def test_fp32_report_vs_fp64():
    cfg = wl.TREE_E8K3
    weights = wl.make_weights(cfg, wl.WEIGHT_SEEDS["tree-e8k3"])
    ue = wl.make_ue_state(cfg.num_ue, wl.ue_seed(7))
    for force_level in (True, False):
        alloc, logits, path = _codebook(cfg, weights, None, ue, force_level)
        rep = parity.compare(cfg, weights, ue, alloc, logits, logit_tol=1e-4)
        rep.check(f"fp32 {path} vs FP64 oracle", exact=True)
        REPORT[f"tree-e8k3/fp32/{path}"] = {"vs_fp64_oracle": rep.as_dict()}
    with open(os.path.join(REPORT_DIR, "precision_report.json"), "w") as f:
        json.dump(REPORT, f, indent=1)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_stress_shape_sampled(prec):
    """The E=16, K=4, 66->512^3->16 actor at full tree size, checked on a
    sample of nodes recomputed one by one from the GPU's parent states."""
    cfg = wl.STRESS_E16K4.with_precision(prec)
    seed = wl.WEIGHT_SEEDS["stress-e16k4"]
    weights = wl.make_weights(cfg, seed)
    act = SCALES[f"stress-e16k4/{seed}"] if prec == "fp8" else None
    ue = wl.make_ue_state(cfg.num_ue, wl.ue_seed(8))
    alloc, logits, path = _codebook(cfg, weights, act, ue, True)
    parity.check_invariants(cfg, ue, alloc)
    nodes = wl.sample_nodes(cfg, 400, seed=9)
    rep = parity.compare(cfg, weights, ue, alloc, logits, nodes=nodes, precision=prec, act_scale=act,
                         logit_tol=SAME_PREC_TOL[prec])
    rep.check(f"{prec} stress sampled", exact=False)
