"""Benchmark of the puncturing-codebook builder on one MI355X.

One step = one whole codebook build (every level of the arrival tree: feature
assembly, actor MLP on MFMA, softmax, capped split, largest remainder) for the
E=8, K=3, M=7 tree with a 34->256->256->8 actor (21,845 nodes, 16,383 actor
evaluations), one codebook per launch, UE state already resident in HBM.

Prints ONE JSON line. `value` is codebook nodes per second of the FP32 build
(the headline precision); the same line carries the build-latency
distribution against the 125 us numerology-3 slot (device-resident and
host-inclusive, i.e. s(t) in host memory -> codebook in pinned host memory),
the BF16 and FP8 legs, the roofline of the dominant kernel and the FP64 CPU
oracle's rate on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2506_00167_amd import workload as wl  # noqa: E402

PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
SLOT_US = 125.0
WORKLOAD = "tree-e8k3"


# Sources each kernel path is compiled from: HBM traffic measured on them is
# reported only while they are unchanged.
KERNEL_SOURCES = {
    "subtree": ["kernels_subtree.hip", "cyrus_regmlp.h", "cyrus_device.h", "cyrus_internal.h"],
    "level": ["kernels_level.hip", "cyrus_device.h", "cyrus_internal.h"],
}


def code_tokens(src: str) -> str:
    """C++/HIP source with comments removed and whitespace collapsed: what the
    compiler sees, so that comment edits keep a measurement valid."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_hash(kernel: str = "subtree") -> str:
    """Hash of the code (comments and whitespace aside) of a kernel's sources."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        h.update(code_tokens(open(os.path.join(ROOT, "paper_2506_00167_amd", "csrc", name)).read()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, precision: str):
    """HBM bytes per launch measured with rocprofv3 counters, if the summary
    was taken on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    entry = data.get(f"{kernel}/{WORKLOAD}/{precision}")
    if not entry or kernel not in KERNEL_SOURCES or entry.get("source_hash") != kernel_source_hash(kernel):
        return None
    return entry.get("bytes_per_launch")


def fp8_act_scales(name: str, seed: int):
    path = os.path.join(ROOT, "tests", "golden", "fp8_act_scales.json")
    data = json.load(open(path))
    return data[f"{name}/{seed}"]


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def run_leg(precision: str, steps: int, warmup: int, latency_builds: int, stream, workload: str = WORKLOAD,
            options=()):
    """options: "hh" (Huntington-Hill rounding), "gaussian" (the Gaussian policy head)."""
    import torch
    from paper_2506_00167_amd import cyrus

    cfg = wl.WORKLOADS[workload].with_precision(precision)
    if "hh" in options:
        cfg = cfg.with_rounding("hh")
    if "gaussian" in options:
        cfg = cfg.with_head("gaussian")
    seed = wl.WEIGHT_SEEDS[workload]
    weights = wl.make_weights(cfg, seed)
    act = fp8_act_scales(workload, seed) if precision == "fp8" else None
    cb = cyrus.Codebook(cfg, weights, act_scale=act, stream=stream)
    cb.set_rng(0x5EED, 1)
    ues = [wl.make_ue_state(cfg.num_ue, wl.ue_seed(i)) for i in range(64)]
    ue_dev = [cyrus.ue_device_tensor(u) for u in ues]
    torch.cuda.synchronize()

    # throughput: back-to-back builds, device-resident inputs, one event pair
    # on the build stream around the whole timed region
    for i in range(warmup):
        cb.build_device(ue_dev[i % 64])
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for i in range(steps):
        cb.build_device(ue_dev[i % 64])
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_us = start.elapsed_time(end) * 1e3 / steps

    # per-build device time (an event pair around each build, so each sample
    # also holds that build's dispatch latency)
    n_ev = min(steps, 500)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_ev)]
    for i in range(n_ev):
        ev[i][0].record(stream)
        cb.build_device(ue_dev[i % 64])
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    dev_us = np.array([a.elapsed_time(b) * 1e3 for a, b in ev])

    # latency: one build at a time, host clock around enqueue + completion
    lat_dev, lat_host = [], []
    for i in range(latency_builds):
        t = time.perf_counter()
        cb.build_device(ue_dev[i % 64])
        cb.wait()
        lat_dev.append((time.perf_counter() - t) * 1e6)
    for i in range(latency_builds):
        u = ues[i % 64]
        t = time.perf_counter()
        cb.build(u)
        cb.wait()
        lat_host.append((time.perf_counter() - t) * 1e6)
    path = cb.kernel_path
    cb.close()

    # the subtree kernel multiplies the static inputs once per launch; the
    # level kernel multiplies the full input row of every node
    flops = cfg.flops_per_codebook_folded if path == "subtree" else cfg.flops_per_codebook
    achieved = flops / (avg_us * 1e-6) / 1e12
    return {
        "workload": workload,
        "options": list(options),
        "precision": precision,
        "kernel": f"{path}",
        "nodes_per_s": cfg.num_nodes * steps / wall,
        "evals_per_s": cfg.num_evals * steps / wall,
        "ms_per_step": wall / steps * 1e3,
        "device_us_mean": avg_us,
        "device_us_per_build_event_p50": pct(dev_us, 50),
        "device_us_per_build_event_p99": pct(dev_us, 99),
        "latency_device_resident_us": {"p50": pct(lat_dev, 50), "p99": pct(lat_dev, 99),
                                       "p99.9": pct(lat_dev, 99.9), "max": float(np.max(lat_dev)),
                                       "misses_over_125us": int(np.sum(np.asarray(lat_dev) > SLOT_US)),
                                       "builds": latency_builds},
        "latency_host_inclusive_us": {"p50": pct(lat_host, 50), "p99": pct(lat_host, 99),
                                      "p99.9": pct(lat_host, 99.9), "max": float(np.max(lat_host)),
                                      "misses_over_125us": int(np.sum(np.asarray(lat_host) > SLOT_US)),
                                      "builds": latency_builds},
        "achieved_tflops": achieved,
        "peak_tflops": PEAK_TFLOPS[precision],
        "mfma_frac": achieved / PEAK_TFLOPS[precision],
        "flops_per_launch": flops,
    }


def critic_leg(steps: int, warmup: int, stream):
    """The Near-RT RIC critic pass (H = 256 samples x M = 7 steps, actor with the
    Gaussian head and four 2 x 256 critics, FP32), timed with one event pair."""
    import torch
    from paper_2506_00167_amd import cyrus

    cfg = wl.CRITIC_RIC
    actor, q, qt = wl.make_critic_weights(cfg, 7)
    cr = cyrus.Critic(cfg, actor, q, qt, stream=stream)
    batch = cyrus.critic_batch_to_device(wl.make_critic_batch(cfg, 8))
    torch.cuda.synchronize()
    for i in range(warmup):
        cr.evaluate(batch, 1, i)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for i in range(steps):
        cr.evaluate(batch, 1, i)
    end.record(stream)
    torch.cuda.synchronize()
    us = start.elapsed_time(end) * 1e3 / steps
    cr.close()
    tflops = cfg.flops / (us * 1e-6) / 1e12
    return {"workload": f"critic pass H={cfg.num_samples} M={cfg.num_minislots} E={cfg.num_ue}, "
                        f"actor {cfg.actor_dims}, critics {cfg.critic_dims}, fp32",
            "us_per_pass": us, "rows_per_s": cfg.rows / (us * 1e-6), "flops_per_pass": cfg.flops,
            "achieved_tflops": tflops, "mfma_frac": tflops / PEAK_TFLOPS["fp32"]}


def gemm_peak(dtype: str, n: int = 8192, reps: int = 10) -> float:
    """Dense TFLOP/s of one large n x n x n torch matmul (the ROCm GEMM
    library) in `dtype` on this GPU: a measured ceiling beside the datasheet
    peak, as context for the roofline fractions."""
    import torch

    dt = {"fp32": torch.float32, "bf16": torch.bfloat16}[dtype]
    g = torch.Generator(device="cuda").manual_seed(1)
    a = torch.randn(n, n, device="cuda", dtype=dt, generator=g)
    b = torch.randn(n, n, device="cuda", dtype=dt, generator=g)
    for _ in range(2):
        torch.matmul(a, b)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        torch.matmul(a, b)
    end.record()
    torch.cuda.synchronize()
    return 2.0 * n ** 3 * reps / (start.elapsed_time(end) * 1e-3) / 1e12


def cpu_baseline(seconds: float):
    """The FP64 oracle, single-threaded, on whole codebooks of the same
    workload until `seconds` of CPU work have been spent."""
    import oracle

    cfg = wl.WORKLOADS[WORKLOAD]
    weights = wl.make_weights(cfg, wl.WEIGHT_SEEDS[WORKLOAD])
    actor = oracle.Actor(weights)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        oracle.build_tree(cfg, weights, wl.make_ue_state(cfg.num_ue, wl.ue_seed(n)), actor=actor)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": cfg.num_nodes * n / dt, "unit": "nodes/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} whole {WORKLOAD} codebooks (FP64, single thread), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--latency-builds", type=int, default=2000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--legs", default="fp32,bf16,fp8")
    ap.add_argument("--context-legs",
                    default="tiny-e4k2/fp32,paper-depth1/fp32,tree-e8k3/fp32+hh,tree-e8k3/fp32+gaussian",
                    help="other workloads timed the same way (WORKLOAD/PRECISION[+OPTION...], comma separated: "
                         "options hh, gaussian), reported as context")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-critic", action="store_true")
    ap.add_argument("--no-gemm-peak", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the codebook build of one cell fits one MI355X and the library has "
              f"no multi-GPU path (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2506_00167_amd import cyrus

    cyrus.lib()  # fail loudly if the HIP library is missing
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    legs = {}
    for prec in args.legs.split(","):
        legs[prec] = run_leg(prec, args.steps, args.warmup, args.latency_builds, stream)
        print(f"[bench] {prec}: {legs[prec]['nodes_per_s']:.4g} nodes/s, device {legs[prec]['device_us_mean']:.1f} us, "
              f"p99 host {legs[prec]['latency_host_inclusive_us']['p99']:.1f} us", file=sys.stderr, flush=True)
    context = {}
    for item in filter(None, args.context_legs.split(",")):
        name, rest = item.split("/")
        prec, *opts = rest.split("+")
        context[item] = run_leg(prec, args.steps, args.warmup, args.latency_builds, stream, workload=name,
                                options=tuple(opts))
        print(f"[bench] context {item}: {context[item]['nodes_per_s']:.4g} nodes/s, device "
              f"{context[item]['device_us_mean']:.1f} us, p99 host "
              f"{context[item]['latency_host_inclusive_us']['p99']:.1f} us", file=sys.stderr, flush=True)
    critic = critic_leg(max(10, args.steps // 10), 5, stream) if not args.no_critic else None
    if critic:
        print(f"[bench] critic pass: {critic['us_per_pass']:.1f} us, {critic['achieved_tflops']:.1f} TFLOP/s",
              file=sys.stderr, flush=True)
    measured = {}
    if not args.no_gemm_peak:
        for dt in ("fp32", "bf16"):
            measured[dt] = gemm_peak(dt)
        print(f"[bench] 8192^3 torch matmul: fp32 {measured['fp32']:.1f}, bf16 {measured['bf16']:.1f} TFLOP/s",
              file=sys.stderr, flush=True)
    head = legs["fp32"]
    cfg = wl.WORKLOADS[WORKLOAD]
    out = {
        "metric": "codebook nodes/sec and p99 build latency vs 125us slot, BF16 vs FP32",
        "value": head["nodes_per_s"],
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}: E=8 K=3 M=7 actor 34->256->256->8, one codebook per launch, "
                               f"{cfg.num_nodes} nodes, {cfg.num_evals} evaluations",
                   "nodes": cfg.num_nodes, "evals": cfg.num_evals, "parallelism": "single GPU"},
        "p99_build_latency_us": head["latency_device_resident_us"]["p99"],
        "p99_build_latency_host_inclusive_us": head["latency_host_inclusive_us"]["p99"],
        "slot_us": SLOT_US,
        "roofline": {
            "bound": "mfma",
            "kernel": head["kernel"],
            "achieved": head["achieved_tflops"],
            "peak": PEAK_TFLOPS["fp32"],
            "unit": "TFLOP/s",
            "frac": head["mfma_frac"],
            "traffic": load_traffic(head["kernel"], "fp32"),
            "flops_per_launch": head["flops_per_launch"],
            "avg_launch_us": head["device_us_mean"],
            "measured_peak": measured.get("fp32"),
            "frac_of_measured_peak": head["achieved_tflops"] / measured["fp32"] if measured else None,
        },
        "gemm_tflops_measured": measured or None,
        "legs": legs,
        "context_legs": context,
        "critic": critic,
    }
    if "bf16" in legs:
        out["bf16_vs_fp32_speedup"] = legs["bf16"]["nodes_per_s"] / head["nodes_per_s"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
