"""Stress workload: 32 cells, each an E=16, K=4, M=7 tree (97,656 nodes,
78,124 actor evaluations) with a 66->512->512->512->16 actor in FP8 (E4M3
weights and activations, power-of-two per-tensor scales, FP32 accumulation),
all 32 built together: one persistent batched launch per level.

CLI: python -m paper_2506_00167_amd.stress [--iters N]
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import cyrus
from . import workload as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCALES = os.path.join(ROOT, "tests", "golden", "fp8_act_scales.json")
CELLS = 32
PEAK_FP8_TFLOPS = 5000.0


def make_cells(n: int = CELLS, precision: str = "fp8", stream=None, export_logits: bool = False):
    scales = json.load(open(SCALES))
    cfg = wl.STRESS_E16K4.with_precision(precision)
    base = wl.WEIGHT_SEEDS["stress-e16k4"]
    cells, ues = [], []
    for j in range(n):
        act = scales[f"stress-e16k4/{base + j}"] if precision == "fp8" else None
        cells.append(cyrus.Codebook(cfg, wl.make_weights(cfg, base + j), act_scale=act, force_level=True,
                                    export_logits=export_logits, stream=stream))
        ues.append(cyrus.ue_device_tensor(wl.make_ue_state(cfg.num_ue, 5_000_000 + j)))
    return cfg, cells, ues


def run(iters: int = 20, warmup: int = 3, precision: str = "fp8"):
    import torch
    stream = torch.cuda.Stream()
    cfg, cells, ues = make_cells(precision=precision, stream=stream)
    torch.cuda.synchronize()
    for _ in range(warmup):
        cyrus.build_batch_device(cells, ues, stream)
    torch.cuda.synchronize()
    times = []
    for _ in range(iters):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        cyrus.build_batch_device(cells, ues, stream)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b) * 1e3)
    t = float(np.median(times))
    flops = CELLS * cfg.flops_per_codebook
    out = {"workload": f"stress-e16k4 x{CELLS} cells, {precision}", "batch_us_median": t,
           "batch_us_min": float(np.min(times)), "nodes_per_s": CELLS * cfg.num_nodes / (t * 1e-6),
           "evals_per_s": CELLS * cfg.num_evals / (t * 1e-6), "tflops": flops / (t * 1e-6) / 1e12,
           "flops_per_batch": flops}
    if precision == "fp8":
        out["mfma_frac"] = out["tflops"] / PEAK_FP8_TFLOPS
    for c in cells:
        c.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--precision", default="fp8")
    args = ap.parse_args()
    cyrus.lib()
    print(json.dumps(run(args.iters, precision=args.precision)))


if __name__ == "__main__":
    main()
