"""Pins of the oracle's feature vector, actor forward pass and number formats.

- The forward pass reduces to a library routine: numpy float64 matrix products
  with ReLU must agree with the oracle's loops to rounding.
- Hand-set weights with known outputs.
- bfloat16 / E4M3 rounding agree with torch's own casts (round to nearest
  even), and saturation at 448 is checked by hand.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_00167_amd import workload as wl


def _np_forward(weights, x):
    h = np.asarray(x, dtype=np.float64)
    for i, (w, b) in enumerate(weights):
        h = w.astype(np.float64) @ h + b.astype(np.float64)
        if i + 1 < len(weights):
            h = np.maximum(h, 0.0)
    return h


def test_features_layout_by_hand():
    ue = wl.UEState(rb=np.array([8, 32], np.int32), mcs=np.array([0, 27], np.int32),
                    sinr_db=np.array([16.0, -4.0], np.float32))
    x = oracle.features(ue, [3, 10], tau=5, k=2)
    assert x.tolist() == [8 / 32, 1.0, 0.0, 27 / 32, 0.5, -0.125, 3 / 64, 10 / 64, 5 / 8, 2 / 8]


@pytest.mark.parametrize("hidden", [(256, 256), (64,), (32, 48, 16)])
def test_mlp_matches_numpy(hidden):
    cfg = wl.TreeConfig(num_ue=5, max_arrival=2, hidden=hidden)
    weights = wl.make_weights(cfg, seed=11)
    rng = np.random.default_rng(5)
    actor = oracle.Actor(weights)
    for _ in range(20):
        x = rng.normal(0, 1, size=cfg.d_in)
        z = oracle.mlp(weights, x, actor=actor)
        ref = _np_forward(weights, x)
        assert np.allclose(z, ref, rtol=1e-12, atol=1e-12)


def test_mlp_bias_only_output():
    cfg = wl.TreeConfig(num_ue=3, max_arrival=2, hidden=(8,))
    weights = [(np.zeros((8, cfg.d_in), np.float32), np.ones(8, np.float32)),
               (np.zeros((3, 8), np.float32), np.array([0.5, -1.0, 2.0], np.float32))]
    z = oracle.mlp(weights, np.ones(cfg.d_in))
    assert z.tolist() == [0.5, -1.0, 2.0]


def test_relu_only_on_hidden_layers():
    # identity-like weights: a negative input survives the output layer only
    w1 = np.zeros((2, 2), np.float32)
    w1[0, 0] = 1.0
    w1[1, 1] = 1.0
    weights = [(w1, np.zeros(2, np.float32)), (np.eye(2, dtype=np.float32), np.array([-3.0, 0.0], np.float32))]
    # d_in = 2 is not a tree shape; the MLP itself does not care
    z = oracle.mlp(weights, [-1.0, 2.0])
    assert z.tolist() == [-3.0, 2.0]


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(6)
    vals = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e-3, 500), rng.normal(0, 300, 500)])
    vals = vals.astype(np.float32).astype(np.float64)
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle.round_bf16(v) for v in vals])
    assert np.array_equal(got, ref)


def test_e4m3_rounding_matches_torch_and_saturates():
    rng = np.random.default_rng(7)
    vals = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 0.01, 500), rng.uniform(-460, 460, 500)])
    vals = vals.astype(np.float32).astype(np.float64)
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = np.array([oracle.round_e4m3(v) for v in vals])
    assert np.array_equal(got, ref)
    assert oracle.round_e4m3(1000.0) == 448.0 and oracle.round_e4m3(-1e9) == -448.0
    assert oracle.round_e4m3(2.0 ** -9) == 2.0 ** -9          # smallest subnormal
    assert oracle.round_e4m3(2.0 ** -10) == 0.0               # tie to even -> 0
    assert oracle.round_e4m3(1.0625) == 1.0                   # tie to even (1.0 vs 1.125)
    assert oracle.round_e4m3(1.1875) == 1.25


def test_e4m3_weight_scale_is_tight_power_of_two():
    for amax in [0.05, 0.3, 1.0, 448.0, 449.0, 3000.0]:
        s = oracle.e4m3_weight_scale(np.array([amax, -amax / 3], np.float32))
        assert s == 2.0 ** round(np.log2(s))
        a32 = float(np.float32(amax))
        assert a32 / s <= 448.0 < a32 / (s / 2)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_quantized_forward_matches_torch_rounding(prec):
    cfg = wl.TreeConfig(num_ue=4, max_arrival=2, hidden=(64, 32))
    weights = wl.make_weights(cfg, seed=12)
    rng = np.random.default_rng(8)
    act = np.array([2.0 ** -6, 2.0 ** -5, 2.0 ** -4])
    actor = oracle.Actor(weights, prec, act if prec == "fp8" else None)
    tdt = torch.bfloat16 if prec == "bf16" else torch.float8_e4m3fn

    def q(v, scale=1.0):
        t = torch.tensor(np.asarray(v, np.float64) / scale, dtype=torch.float64)
        # cast through float32 is exact for these magnitudes except at ties of
        # the float32 rounding, which random inputs do not hit
        return t.to(torch.float32).to(tdt).to(torch.float64).numpy() * scale

    for _ in range(10):
        x = rng.normal(0, 1, size=cfg.d_in)
        z = oracle.mlp(weights, x, actor=actor)
        h = x
        for i, (w, b) in enumerate(weights):
            if prec == "fp8":
                sw = oracle.e4m3_weight_scale(w)
                hq, wq = q(h, act[i]), q(w, sw)
            else:
                hq, wq = q(h), q(w)
            h = wq @ hq + b.astype(np.float64)
            if i + 1 < len(weights):
                h = np.maximum(h, 0.0)
        assert np.allclose(z, h, rtol=1e-12, atol=1e-12)
