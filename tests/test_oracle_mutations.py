"""The oracle's pins must catch plausible mistakes.

Each case below plants one mistake in a copy of the oracle's C source (a
dropped term, a wrong sign, index or scale, a transposed operand, a broken tie
rule), compiles it to a temporary library and runs the pin tests against it.
At least one pin must fail for every mutant. The mistakes live only in the
temporary copies; the oracle itself is untouched.
"""
import contextlib
import os

import pytest

import oracle
from tests import test_oracle_alloc as ta
from tests import test_oracle_critic as tc
from tests import test_oracle_gaussian as tg
from tests import test_oracle_hh as th
from tests import test_oracle_mlp as tm
from tests import test_oracle_tree as tt

SRC = open(oracle._SRC).read()

MUTANTS = {
    "feature c scale": ("x[3 * E + e] = c[e] / 64.0;", "x[3 * E + e] = c[e] / 32.0;"),
    "feature tau/k swapped": ("x[4 * E] = tau / 8.0;\n    x[4 * E + 1] = k / 8.0;",
                              "x[4 * E] = k / 8.0;\n    x[4 * E + 1] = tau / 8.0;"),
    "bias dropped": ("acc += (double)f->b[l][o];", "acc += 0.0;"),
    "relu on output layer": ("g[o] = (l + 1 < f->num_layers && acc < 0.0) ? 0.0 : acc;",
                             "g[o] = (acc < 0.0) ? 0.0 : acc;"),
    "transposed weights": ("acc += quantize((double)wrow[i], f->precision, s_w) * h[i];",
                           "acc += quantize((double)f->w[l][(int64_t)i * out + o], f->precision, s_w) * h[i];"),
    "softmax sign": ("p[e] = exp(d);", "p[e] = exp(-d);"),
    "softmax not normalised": ("p[e] /= sum;", "p[e] /= 1.0;"),
    "capped demand not removed": ("rem -= R[e];", "rem -= 0;"),
    "cap test reversed": ("s * p[e] >= (double)R[e]", "s * p[e] <= (double)R[e]"),
    "demand ignores RBs per arrival": ("int64_t demand = (int64_t)U * k;", "int64_t demand = k;"),
    "tie to higher index": ("if (frac > best_frac) {", "if (frac >= best_frac) {"),
    "cap ignored in rounding": ("if (picked[e] || a[e] >= R[e])", "if (picked[e])"),
    "smallest remainder first": ("double frac = x[e] - floor(x[e]);", "double frac = 1.0 - (x[e] - floor(x[e]));"),
    "wrong parent index": ("parent = poff + i / (K + 1);", "parent = poff + i / K;"),
    "state not carried": ("state[node * E + e] = c_in[e] + a[e];", "state[node * E + e] = a[e];"),
    "arrival digit off by one": ("const int32_t k = (int32_t)(i % (K + 1));",
                                 "const int32_t k = (int32_t)((i + 1) % (K + 1));"),
    "level offset": ("return (ipow64(K + 1, tau) - 1) / K;", "return ipow64(K + 1, tau) / K;"),
    "bf16 mantissa": ("return round_sig(v, 8, -126 - 7);", "return round_sig(v, 7, -126 - 7);"),
    "e4m3 saturation": ("if (r > 448.0)\n        r = 448.0;", "if (r > 480.0)\n        r = 480.0;"),
    "rollout state": ("            c[e] += a[e];", "            c[e] += 0;"),
    "hh arithmetic-mean divisor": ("x[e] / sqrt((double)a[e] * (double)(a[e] + 1));",
                                   "x[e] / ((double)a[e] + 0.5);"),
    "hh first unit not guaranteed": ("a[e] == 0 ? INFINITY :", "a[e] == 0 ? x[e] :"),
    "hh tie to smaller share": ("(pr == best_pr && x[e] > x[best])", "(pr == best_pr && x[e] < x[best])"),
    "hh cap ignored": ("if (!(x[e] > 0.0) || a[e] >= R[e])\n                continue;\n            const double pr",
                       "if (!(x[e] > 0.0))\n                continue;\n            const double pr"),
    "philox round constant": ("(uint64_t)0xCD9E8D57u * c2;", "(uint64_t)0xCD9E8D55u * c2;"),
    "philox key schedule": ("k1 += 0xBB67AE85u;", "k1 += 0x9E3779B9u;"),
    "box-muller radius": ("return sqrt(-2.0 * log(u1)) * cos(two_pi * u2);", "return sqrt(-log(u1)) * cos(two_pi * u2);"),
    "normal counter ignores the UE": ("const uint32_t ctr[4] = {(uint32_t)node, (uint32_t)e,",
                                      "const uint32_t ctr[4] = {(uint32_t)node, (uint32_t)0,"),
    "log-sigma clamp": ("return ls < -20.0 ? -20.0 : (ls > 2.0 ? 2.0 : ls);", "return ls < -20.0 ? -20.0 : ls;"),
    "share map without the half": ("z[e] = u >= 0.0 ? -log1p(exp(-2.0 * u)) : 2.0 * u - log1p(exp(2.0 * u));",
                                   "z[e] = u >= 0.0 ? -log1p(exp(-u)) : u - log1p(exp(u));"),
    "rollout node counter": ("oracle_level_offset(K, tau) + i, tau, k, a, z, NULL, amax);",
                             "oracle_level_offset(K, tau) + i / (K + 1), tau, k, a, z, NULL, amax);"),
    "log-density Jacobian sign": ("lp += -0.5 * d * d - ls - half_log_two_pi - log_jac;",
                                  "lp += -0.5 * d * d - ls - half_log_two_pi + log_jac;"),
    "log-density missing log sigma": ("lp += -0.5 * d * d - ls - half_log_two_pi - log_jac;",
                                      "lp += -0.5 * d * d - half_log_two_pi - log_jac;"),
    "target takes the larger critic": ("(qt[0] < qt[1] ? qt[0] : qt[1])", "(qt[0] > qt[1] ? qt[0] : qt[1])"),
    "entropy term added": ("- cfg->entropy_coef * lp);", "+ cfg->entropy_coef * lp);"),
    "target from the same step": ("const int64_t nrow = row + 1;", "const int64_t nrow = row;"),
    "loss not averaged": ("loss[i] = sq[i] / ((double)H * M);", "loss[i] = sq[i] / (double)H;"),
    "lr margin always zero": ("return 0.5 * (rem[r - 1] - rem[r]);", "return 0.0;"),
    "lr margin the whole gap": ("return 0.5 * (rem[r - 1] - rem[r]);", "return rem[r - 1] - rem[r];"),
    "lr margin counts floor crossings": ("return 0.5 * (rem[r - 1] - rem[r]);",
                                         "return fmin(0.5 * (rem[r - 1] - rem[r]), fmin(rem[r - 1], 1.0 - rem[0]));"),
    "lr margin infinite on integer shares": ("    if (r == 0)\n        return 0.5;",
                                             "    if (r == 0)\n        return INFINITY;"),
    "lr margin remainders ascending": ("while (j >= 0 && rem[j] < v)", "while (j >= 0 && rem[j] > v)"),
    "hh margin without the first-unit term": (
        "        if (x[i] < m) /* a first unit is owed only to a positive share */\n            m = x[i];\n", ""),
    "hh margin one-sided": ("double d = (x[i] / hi - x[j] / hj) / (1.0 / hi + 1.0 / hj);",
                            "double d = (x[i] / hi - x[j] / hj) * hi;"),
    "hh margin ignores the cap of the rising share": ("            if (x[j] + d > (double)R[j])\n", "            if (0)\n"),
}

PINS = [
    ta.test_table6_rp_first_packet,
    lambda: ta.test_hand_split_uncapped(2, 3, [2, 2, 1, 1]),
    ta.test_hand_split_cap_and_tie,
    ta.test_hand_demand_above_capacity,
    ta.test_softmax_properties,
    ta.test_capped_scale_kkt,
    ta.test_largest_remainder_tie_goes_to_lower_index,
    ta.test_margin_hand_cases,
    lambda: ta.test_margin_is_safe_and_tight("split"),
    lambda: ta.test_margin_is_safe_and_tight("integer"),
    tm.test_features_layout_by_hand,
    lambda: tm.test_mlp_matches_numpy((32, 48, 16)),
    tm.test_relu_only_on_hidden_layers,
    tm.test_bf16_rounding_matches_torch,
    tm.test_e4m3_rounding_matches_torch_and_saturates,
    tt.test_node_counts_by_enumeration,
    lambda: tt.test_tree_equals_brute_force_rollouts(False),
    lambda: tt.test_invariants_tiny_workload(True),
    tt.test_depth_one_is_the_papers_codebook,
    th.test_matches_divisor_form_random,
    th.test_hand_case_differs_from_largest_remainder,
    th.test_hand_case_cap_and_ties,
    th.test_tie_goes_to_larger_share_then_lower_index,
    th.test_zero_share_and_cap_never_receive,
    th.test_margin_is_a_safe_distance,
    th.test_margin_is_tight_on_a_swap,
    th.test_margin_first_units,
    tg.test_philox_known_answers,
    tg.test_normal_is_standard,
    tg.test_normal_depends_on_every_key_part,
    tg.test_head_matches_tanh_on_the_same_draws,
    tg.test_head_clamps_log_sigma,
    lambda: tg.test_gaussian_tree_equals_rollouts("lr"),
    tc.test_policy_density_integrates_to_one,
    tc.test_policy_density_matches_scipy,
    tc.test_sample_is_the_heads_draw_through_tanh,
    tc.test_hand_set_critics_give_the_closed_form_target_and_loss,
    tc.test_critic_forward_matches_numpy,
]


@contextlib.contextmanager
def _swapped(lib_obj):
    saved = oracle._lib
    oracle._lib = lib_obj
    try:
        yield
    finally:
        oracle._lib = saved


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, f"mutation site of '{name}' not found exactly once"
    src = tmp_path / "mutant.c"
    src.write_text(SRC.replace(old, new))
    so = oracle.compile_oracle(str(tmp_path / "libmutant.so"), str(src))
    caught = []
    with _swapped(oracle._load(so)):
        for pin in PINS:
            try:
                pin()
            except (AssertionError, ValueError):
                caught.append(getattr(pin, "__name__", "lambda"))
    assert caught, f"no pin catches the planted mistake '{name}'"
