"""Writes fp8_act_scales.json: the static per-layer input scales of the FP8
actor variants, calibrated with the FP64 oracle only.

For each workload and weight seed, random arrival sequences are rolled out by
the oracle on calibration UE states (seeds that no test or benchmark uses),
the largest |input| of every layer is recorded, and the scale is the smallest
power of two s with 2 * amax / s <= 448 (E4M3's largest finite value), i.e.
one octave of headroom for states the calibration did not visit.

Run from the repository root: python tests/golden/make_fp8_scales.py
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2506_00167_amd import workload as wl  # noqa: E402

CAL_UE_SEEDS = [3_000_000 + i for i in range(4)]
SEQUENCES_PER_STATE = 64


def calibrate(cfg, weights):
    actor = oracle.Actor(weights)
    amax = np.zeros(len(weights), dtype=np.float64)
    for s in CAL_UE_SEEDS:
        ue = wl.make_ue_state(cfg.num_ue, s)
        for seq in wl.random_sequences(cfg, SEQUENCES_PER_STATE, seed=s + 17):
            seq = np.maximum(seq, 1)  # every mini-slot evaluated
            oracle.rollout(cfg, weights, ue, seq, actor=actor, amax=amax)
    return [2.0 ** math.ceil(math.log2(2.0 * a / 448.0)) for a in amax]


def main():
    out = {}
    jobs = [("tree-e8k3", wl.WEIGHT_SEEDS["tree-e8k3"])]
    jobs += [("stress-e16k4", wl.WEIGHT_SEEDS["stress-e16k4"] + j) for j in range(32)]
    for name, seed in jobs:
        cfg = wl.WORKLOADS[name]
        out[f"{name}/{seed}"] = calibrate(cfg, wl.make_weights(cfg, seed))
        print(name, seed, out[f"{name}/{seed}"], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp8_act_scales.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
