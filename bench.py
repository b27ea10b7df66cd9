"""Benchmark of the puncturing-codebook builder on one MI355X.

One step = one whole codebook build (every level of the arrival tree: feature
assembly, actor MLP on MFMA, softmax, capped split, largest remainder) for the
E=8, K=3, M=7 tree with a 34->256->256->8 actor (21,845 nodes, 16,383 actor
evaluations), one codebook per launch, UE state already resident in HBM.

Prints ONE JSON line. `value` is codebook nodes per second of the FP32 build
(the headline precision); the same line carries the build-latency
distribution against the 125 us numerology-3 slot (host-inclusive, i.e. s(t)
in host memory -> codebook in pinned host memory, as the headline p99; and
device-resident), the BF16 and FP8 legs, the E=4 K=2 tree and other context
legs, the 32-cell FP8 stress batch, the continuous-batching serving stream,
the roofline of the dominant kernel and the FP64 CPU oracle's rate on a
bounded sample (one thread and all threads), with each precision's logit
error and allocation-disagreement rate against that oracle.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import gc
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
    "subtree": ["kernels_subtree.hip", "cyrus_subtree.h", "cyrus_regmlp.h", "cyrus_device.h", "cyrus_internal.h"],
    "level": ["kernels_level.hip", "cyrus_mlp.h", "cyrus_serve.h", "cyrus_subtree.h", "cyrus_regmlp.h",
              "cyrus_device.h", "cyrus_internal.h"],
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


PROFILE_TRACES = {
    ("subtree", "fp32"): "subtree_kernel_tree-e8k3_fp32_trace.txt",
    ("subtree", "bf16"): "subtree_kernel_tree-e8k3_bf16_trace.txt",
    ("subtree", "fp8"): "subtree_kernel_tree-e8k3_fp8_trace.txt",
}


def profiled_kernel_us(kernel: str, precision: str):
    """Average kernel duration of this workload's builds from the committed
    rocprofv3 trace summary, if it was taken on the current kernel sources."""
    name = PROFILE_TRACES.get((kernel, precision))
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_hash: (\w+)", text)
    a = re.search(r"kernel_trace: dispatches=\d+ avg_us=([0-9.]+)", text)
    if not m or not a or m.group(1) != kernel_source_hash(kernel):
        return None
    return float(a.group(1))


def fp8_act_scales(name: str, seed: int):
    path = os.path.join(ROOT, "tests", "golden", "fp8_act_scales.json")
    data = json.load(open(path))
    return data[f"{name}/{seed}"]


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def latency_stats(lat_us):
    """Distribution of one-at-a-time build latencies against the slot, with
    the five slowest samples and their positions in the run."""
    a = np.asarray(lat_us)
    worst = np.argsort(a)[::-1][:5]
    return {"p50": pct(a, 50), "p99": pct(a, 99), "p99.9": pct(a, 99.9), "max": float(a.max()),
            "misses_over_125us": int(np.sum(a > SLOT_US)), "builds": int(a.size),
            "slowest": [[int(i), round(float(a[i]), 1)] for i in worst]}


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

    # latency: one build at a time, host clock around enqueue + completion,
    # a new UE state for every build (seeded, as the throughput states are).
    # Host-inclusive builds (the paper's definition: s(t) in host memory ->
    # codebook in pinned host memory) get their own warm-up, which touches the
    # pinned mirror and the mapped UE staging first; the Python collector is
    # off while timing so that its pauses do not land in a sample.
    lat_ues = [wl.make_ue_state(cfg.num_ue, wl.ue_seed(64 + i)) for i in range(latency_builds)]
    ue_structs = [cyrus.ue_struct(u) for u in lat_ues]
    packed = np.stack([np.concatenate([np.asarray(u.rb, np.int32), np.asarray(u.mcs, np.int32),
                                       np.asarray(u.sinr_db, np.float32).view(np.int32)]) for u in lat_ues])
    lat_dev_ues = torch.from_numpy(packed).to("cuda")  # one row per build, the layout of ue_device_tensor
    torch.cuda.synchronize()
    row_bytes = lat_dev_ues.shape[1] * 4
    for i in range(max(warmup, 1)):
        cb.build(ues[i % 64])
        cb.wait()
    lat_dev, lat_host = [], []
    gc_was = gc.isenabled()
    gc.disable()
    try:
        base = lat_dev_ues.data_ptr()
        for i in range(latency_builds):
            t = time.perf_counter()
            cyrus.cyrus_codebook_build_device(cb.handle, base + i * row_bytes, cb.stream)
            cb.wait()
            lat_dev.append((time.perf_counter() - t) * 1e6)
        for i in range(latency_builds):
            st = ue_structs[i][0]
            t = time.perf_counter()
            cyrus.cyrus_codebook_build(cb.handle, st, cb.stream)
            cb.wait()
            lat_host.append((time.perf_counter() - t) * 1e6)
    finally:
        if gc_was:
            gc.enable()
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
        "latency_device_resident_us": latency_stats(lat_dev),
        "latency_host_inclusive_us": latency_stats(lat_host),
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


def host_cpu_info():
    """Core counts and CPU model of the host the oracle is timed on."""
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return info


def _oracle_rate(workload: str, seconds: float, threads: int):
    """Whole codebooks of `workload` built by the FP64 oracle in `threads`
    host threads (each thread its own codebooks; the oracle's C calls run
    without the interpreter lock) until `seconds` have passed."""
    import concurrent.futures as cf
    import oracle

    cfg = wl.WORKLOADS[workload]
    weights = wl.make_weights(cfg, wl.WEIGHT_SEEDS[workload])
    actor = oracle.Actor(weights)
    ues = [wl.make_ue_state(cfg.num_ue, wl.ue_seed(i)) for i in range(64)]
    t0 = time.perf_counter()

    def worker(tid):
        n = 0
        while time.perf_counter() - t0 < seconds:
            oracle.build_tree(cfg, weights, ues[(tid + n * threads) % 64], actor=actor)
            n += 1
        return n

    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        counts = list(ex.map(worker, range(threads)))
    dt = time.perf_counter() - t0
    n = sum(counts)
    return cfg.num_nodes * n / dt, n, dt


def oracle_agreement(stream):
    """Each precision's C2 codebook against the FP64 oracle on one UE state:
    the largest logit difference at evaluated nodes (conditioned mode: the
    oracle evaluates every node from the GPU's own parent state) and the
    allocation-disagreement rates, conditioned and free-running. FP32
    disagreements are also split at the 1e-6 decision margin."""
    import oracle
    from paper_2506_00167_amd import cyrus

    cfg0 = wl.WORKLOADS[WORKLOAD]
    seed = wl.WEIGHT_SEEDS[WORKLOAD]
    weights = wl.make_weights(cfg0, seed)
    ue = wl.make_ue_state(cfg0.num_ue, wl.ue_seed(0))
    free, _, _ = oracle.build_tree(cfg0, weights, ue)
    K = cfg0.max_arrival
    ev = np.zeros(cfg0.num_nodes, bool)
    for tau in range(1, cfg0.num_minislots + 1):
        off, width = oracle.level_offset(K, tau), (K + 1) ** tau
        ev[off:off + width] = np.arange(width) % (K + 1) != 0
    out = {"workload": WORKLOAD, "ue_seed": wl.ue_seed(0), "reference": "FP64 oracle (exact weights and inputs)"}
    for prec in ("fp32", "bf16", "fp8"):
        cfg = cfg0.with_precision(prec)
        act = fp8_act_scales(WORKLOAD, seed) if prec == "fp8" else None
        cb = cyrus.Codebook(cfg, weights, act_scale=act, export_logits=True, stream=stream)
        cb.build(ue)
        cb.wait()
        alloc, logits = cb.export()
        cb.close()
        c_alloc, c_logits, marg = oracle.eval_conditioned(cfg0, weights, ue, alloc)
        mism = (c_alloc != alloc.astype(np.int32)).any(axis=1) & ev
        fm = (free != alloc).any(axis=1) & ev
        out[prec] = {"max_logit_err": float(np.abs(logits[ev] - c_logits[ev]).max()),
                     "disagreement_rate_conditioned": float(mism.sum() / ev.sum()),
                     "disagreement_rate_free_running": float(fm.sum() / ev.sum()),
                     "conditioned_disagreements": int(mism.sum()),
                     "below_1e-6_margin": int((mism & (marg < 1e-6)).sum()),
                     "evals": int(ev.sum())}
    return out


def cpu_baseline(seconds: float, threads: int, stream):
    """The FP64 oracle as it stands, timed on this host: whole codebooks of
    the headline workload on one thread and on `threads` threads, and of the
    E=4 K=2 workload on one thread. The same leg runs the oracle against each
    precision's GPU codebook (the only place the benchmark loads it)."""
    one, n1, dt1 = _oracle_rate(WORKLOAD, seconds, 1)
    many, nn, dtn = _oracle_rate(WORKLOAD, seconds, threads)
    tiny, nt, dtt = _oracle_rate("tiny-e4k2", min(seconds, 4.0), 1)
    host = host_cpu_info()
    return {"value": many, "unit": "nodes/s", "cores": threads, "kind": "oracle",
            "sample": f"{nn} whole {WORKLOAD} codebooks (FP64) on {threads} threads in {dtn:.1f} s; "
                      f"single thread: {n1} codebooks in {dt1:.1f} s",
            "single_thread_value": one, "host": host,
            "tiny-e4k2_single_thread_value": tiny,
            "tiny-e4k2_sample": f"{nt} whole tiny-e4k2 codebooks in {dtt:.1f} s",
            "precision_vs_oracle": oracle_agreement(stream)}


def stress_leg(iters: int, stream):
    """32 cells of E=16 K=4 M=7 with a 66->512^3->16 FP8 actor, built by one
    batched level launch per level (a persistent grid over every cell's tiles)."""
    import torch
    from paper_2506_00167_amd import cyrus, stress

    cfg, cells, ues = stress.make_cells(stream=stream)
    torch.cuda.synchronize()
    for _ in range(20):
        cyrus.build_batch_device(cells, ues, stream)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(iters):
        cyrus.build_batch_device(cells, ues, stream)
    end.record(stream)
    torch.cuda.synchronize()
    us = start.elapsed_time(end) * 1e3 / iters
    for c in cells:
        c.close()
    n = len(cells)
    flops = n * cfg.flops_per_codebook
    tflops = flops / (us * 1e-6) / 1e12
    return {"workload": f"stress-e16k4 x{n} cells: E=16 K=4 M=7, actor 66->512->512->512->16, fp8, "
                        f"{cfg.num_nodes} nodes per cell",
            "batches": iters, "us_per_batch": us, "nodes_per_s": n * cfg.num_nodes / (us * 1e-6),
            "evals_per_s": n * cfg.num_evals / (us * 1e-6), "flops_per_batch": flops, "achieved_tflops": tflops,
            "mfma_frac": tflops / PEAK_TFLOPS["fp8"]}


def serving_leg(requests: int, stream):
    """Continuous batching of Poisson requests from 64 BF16 cells (E 4..16,
    K 2..4, two hidden layers of 256 or 512) on the resident worker:
    saturation, then a quarter of it, then a pool that holds only a few
    trees, so admission defers."""
    import torch
    from paper_2506_00167_amd import serving

    cells = serving.make_cells(64, stream=stream)
    torch.cuda.synchronize()
    out = {"workload": "64 cells, E U{4..16}, K U{2,3,4}, H {256,512} x2, bf16, Poisson arrivals",
           "engine": "resident worker", "requests": requests}
    eng = serving.default_engine(128, 256, stream=stream, resident=True)
    serving.saturation(eng, cells, serving.make_requests(cells, 200, seed=1))
    sat = serving.saturation(eng, cells, serving.make_requests(cells, requests, seed=2))
    out["saturation"] = sat
    rate = sat["served_req_per_s"]
    arr = wl.poisson_arrivals(0.25 * rate, requests, seed=424242)
    out["load_0.25"] = serving.run_stream(eng, cells, serving.make_requests(cells, requests, seed=3), arr - arr[0])
    eng.close()
    # device pool: the descriptor slots plus room for about two of the
    # largest trees, so that admission has to wait for memory
    biggest = max(c.num_nodes * c.cfg.num_ue for c in cells)
    pool = 3 * biggest + (2 << 20)
    from paper_2506_00167_amd import cyrus
    small = cyrus.Engine(pool, pool + (8 << 20), max_active=128, stream=stream, resident=True)
    arr = wl.poisson_arrivals(0.5 * rate, requests // 2, seed=424243)
    out["small_pool_load_0.5"] = serving.run_stream(small, cells, serving.make_requests(cells, requests // 2, seed=4),
                                                    arr - arr[0])
    out["small_pool_bytes"] = pool
    small.close()
    out["one_request_per_cell_per_slot_req_per_s"] = 8000.0 * len(cells)
    for c in cells:
        c.close()
    return out


# The paper's own timing of the codebook build (Sec. VII): a different
# workload on other hardware, reported beside the leg of the same shape here
# and never used as vs_baseline.
PAPER_TIMING = {
    "codebook_build_us_mean": 94.4,
    "codebook_build_us_max_below": 125.0,
    "tti_samples": 1000,
    "hardware": "DGX Station (NVIDIA V100), TensorFlow",
    "workload": "depth 1 (one mini-slot), E=10, 2 arrival branches, one hidden layer of 128, Gaussian policy "
                "head, Huntington-Hill rounding",
    "timing": "s(t) received -> B*(t) produced",
}


def paper_context(context):
    out = dict(PAPER_TIMING)
    leg = context.get("paper-depth1/fp32+gaussian+hh")
    if leg:
        h = leg["latency_host_inclusive_us"]
        out["here"] = {"leg": "paper-depth1/fp32+gaussian+hh", "kernel": leg["kernel"],
                       "host_inclusive_us_p50": h["p50"], "host_inclusive_us_p99": h["p99"],
                       "host_inclusive_us_max": h["max"], "misses_over_125us": h["misses_over_125us"],
                       "device_us_mean": leg["device_us_mean"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--latency-builds", type=int, default=10000,
                    help="one-at-a-time builds per leg for the latency distribution, a new UE state each")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="seconds of oracle work per CPU-baseline sample (one thread, then all threads)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the all-cores oracle sample (default: the CPUs this process may run on, "
                         "at most 16)")
    ap.add_argument("--no-stress", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--stress-iters", type=int, default=200)
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--legs", default="fp32,bf16,fp8")
    ap.add_argument("--context-legs",
                    default="tiny-e4k2/fp32,paper-depth1/fp32,paper-depth1/fp32+gaussian+hh,tree-e8k3/fp32+hh,"
                            "tree-e8k3/fp32+gaussian",
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
    stress = stress_leg(args.stress_iters, stream) if not args.no_stress else None
    if stress:
        print(f"[bench] stress: {stress['us_per_batch']:.0f} us per 32-cell batch, {stress['nodes_per_s']:.4g} nodes/s, "
              f"{stress['mfma_frac']:.3f} of FP8 peak", file=sys.stderr, flush=True)
    serving_res = serving_leg(args.serving_requests, stream) if not args.no_serving else None
    if serving_res:
        q = serving_res["load_0.25"]
        print(f"[bench] serving: saturation {serving_res['saturation']['served_req_per_s']:.0f} req/s; at 0.25 load "
              f"p50 {q['latency_us']['p50']:.0f} us, p99 {q['latency_us']['p99']:.0f} us, "
              f"{q['misses_over_125us']} of {q['requests']} over 125 us", file=sys.stderr, flush=True)
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
    prof_us = profiled_kernel_us(head["kernel"], "fp32")
    for prec, leg in legs.items():
        pu = profiled_kernel_us(leg["kernel"], prec)
        leg["profiled_kernel_us"] = pu
        leg["mfma_frac_profiled_kernel_time"] = (leg["flops_per_launch"] / (pu * 1e-6) / 1e12 / PEAK_TFLOPS[prec]
                                                 if pu else None)
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
        # the paper's definition: from s(t) received (host memory) until the
        # codebook is produced (pinned host memory)
        "p99_build_latency_us": head["latency_host_inclusive_us"]["p99"],
        "p99_build_latency_device_resident_us": head["latency_device_resident_us"]["p99"],
        "misses_over_125us": head["latency_host_inclusive_us"]["misses_over_125us"],
        "slot_us": SLOT_US,
        "roofline": {
            "bound": "mfma",
            "kernel": head["kernel"],
            "achieved": head["achieved_tflops"],
            "peak": PEAK_TFLOPS["fp32"],
            "unit": "TFLOP/s",
            "frac": head["mfma_frac"],
            "frac_basis": "event pair around the whole timed region / steps (includes dispatch gaps)",
            "traffic": load_traffic(head["kernel"], "fp32"),
            "flops_per_launch": head["flops_per_launch"],
            "avg_launch_us": head["device_us_mean"],
            "profiled_kernel_us": prof_us,
            "frac_profiled_kernel_time": (head["flops_per_launch"] / (prof_us * 1e-6) / 1e12 / PEAK_TFLOPS["fp32"]
                                          if prof_us else None),
            "measured_peak": measured.get("fp32"),
            "frac_of_measured_peak": head["achieved_tflops"] / measured["fp32"] if measured else None,
        },
        "gemm_tflops_measured": measured or None,
        "legs": legs,
        "context_legs": context,
        "paper_context": paper_context(context),
        "critic": critic,
        "stress": stress,
        "serving": serving_res,
    }
    if "bf16" in legs:
        # back-to-back builds, each with its completion event (what a caller
        # sees); and the kernels alone, from the rocprofv3 traces of the same
        # sources (null when they were taken on other sources)
        out["bf16_vs_fp32_speedup"] = legs["bf16"]["nodes_per_s"] / head["nodes_per_s"]
        pb = legs["bf16"].get("profiled_kernel_us")
        out["bf16_vs_fp32_speedup_kernel_time"] = prof_us / pb if prof_us and pb else None
    if not args.no_cpu:
        threads = args.cpu_threads or min(16, len(os.sched_getaffinity(0)))
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, threads, stream)
        print(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.4g} nodes/s on {threads} threads",
              file=sys.stderr, flush=True)
        out["precision_vs_oracle"] = out["cpu_baseline"].pop("precision_vs_oracle")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
