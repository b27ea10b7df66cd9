"""Serving workload: a Poisson stream of codebook requests from many simulated
cells, fed to the continuous-batching engine of libcyrus.

Each cell has its own shape (E UEs, arrival alphabet 0..K, hidden width) and
its own actor weights, resident on the GPU in a Codebook handle. A request is
one TTI of one cell. Latency is measured from the request's scheduled arrival
time to the moment the host observes its codebook in pinned memory, and is
reported against the 125 us slot of numerology 3.

CLI: python -m paper_2506_00167_amd.serving [--requests N] [--loads 0.25,0.5,...]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import cyrus
from . import workload as wl

SLOT_US = 125.0


def make_cells(num_cells: int = 64, seed: int = 424242, device: str = "cuda", stream=None):
    cells = []
    for cfg, wseed in wl.serving_cell_configs(num_cells, seed):
        cells.append(cyrus.Codebook(cfg, wl.make_weights(cfg, wseed), device=device,
                                    stream=stream))
    return cells


def make_requests(cells, n: int, seed: int = 7):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        c = int(rng.integers(0, len(cells)))
        out.append((c, wl.make_ue_state(cells[c].cfg.num_ue, 9_000_000 + i)))
    return out


def default_engine(max_active: int = 64, pool_mib: int = 256, stream=None, levels_per_step: int = 1,
                   resident: bool = False):
    eng = cyrus.Engine(pool_mib << 20, pool_mib << 20, max_active=max_active, stream=stream, resident=resident)
    return eng if resident else eng.set_levels_per_step(levels_per_step)


def run_stream(engine, cells, requests, arrivals_s, keep_results: bool = False, native: bool = True):
    """Submit requests at their arrival times while stepping the engine.
    Returns latency statistics (us), throughput and engine counters.
    native: the library's own request loop (cyrus_engine_run); else a Python
    loop over submit / step / completed / result."""
    n = len(requests)
    if native:
        arr_us = (np.asarray(arrivals_s, dtype=np.float64) - arrivals_s[0]) * 1e6
        lat, outs = engine.run([cells[c] for c, _ in requests], [ue for _, ue in requests], arr_us, keep_results)
        # the span on the loop's own clock: from its start to the last completion
        span_s = float((arr_us + lat).max()) * 1e-6
        return _stats(engine, cells, requests, arrivals_s, lat, span_s + arrivals_s[0], "native",
                      dict(enumerate(outs)) if keep_results else None)
    t0 = time.perf_counter()
    sub_wall = {}
    lat_engine = {}
    results = {}
    i = 0
    idle_steps = 0
    while len(lat_engine) < n:
        now = time.perf_counter() - t0
        while i < n and arrivals_s[i] <= now:
            c, ue = requests[i]
            t = engine.submit(cells[c], ue)
            sub_wall[t] = (i, time.perf_counter() - t0)
            i += 1
        running, waiting = engine.step()
        for t, l in engine.completed():
            lat_engine[t] = l
            r = engine.result(t)
            if keep_results:
                results[sub_wall[t][0]] = r
        if running == 0 and waiting == 0 and i < n and len(lat_engine) == i:
            idle_steps += 1
            while time.perf_counter() - t0 < arrivals_s[i]:
                pass
    wall = time.perf_counter() - t0
    lat = []
    for t, l in lat_engine.items():
        idx, s = sub_wall[t]
        lat.append(l + (s - arrivals_s[idx]) * 1e6)  # count queueing before submit too
    return _stats(engine, cells, requests, arrivals_s, np.array(lat), wall, "python",
                  results if keep_results else None)


def _stats(engine, cells, requests, arrivals_s, lat, wall, loop, results):
    n = len(requests)
    nodes = sum(cells[c].num_nodes for c, _ in requests)
    flops = sum(cells[c].cfg.flops_per_codebook for c, _ in requests)
    span = wall - arrivals_s[0]
    out = {
        "requests": n,
        "offered_req_per_s": n / max(arrivals_s[-1] - arrivals_s[0], 1e-9),
        "served_req_per_s": n / span,
        "nodes_per_s": nodes / span,
        "tflops": flops / span / 1e12,
        "latency_us": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "p99.9": float(np.percentile(lat, 99.9)), "max": float(lat.max()),
                       "mean": float(lat.mean())},
        "misses_over_125us": int((lat > SLOT_US).sum()),
        "request_loop": loop,
        "engine": engine.stats(),
    }
    if results is not None:
        out["results"] = results
    return out


def saturation(engine, cells, requests, native: bool = True):
    """Everything submitted at t = 0: the engine's sustained throughput."""
    return run_stream(engine, cells, requests, np.zeros(len(requests)), native=native)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=64)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--loads", default="0.25,0.5,0.75,0.9")
    ap.add_argument("--max-active", type=int, default=64)
    ap.add_argument("--pool-mib", type=int, default=256)
    ap.add_argument("--level-lag", type=int, default=None,
                    help="resident worker: requests built by level tiles rank as if admitted this many requests "
                         "later (0: first come, first served; default: the library's)")
    ap.add_argument("--python-loop", action="store_true",
                    help="drive the engine from a Python loop instead of the library's cyrus_engine_run")
    ap.add_argument("--levels-per-step", default="0,1,7",
                    help="comma separated engine modes: 0 = the resident worker, 1 = host-stepped iteration-level "
                         "batching, 7 = each host step runs its requests to the end")
    args = ap.parse_args()
    import torch
    cyrus.lib()
    stream = torch.cuda.Stream()
    cells = make_cells(args.cells, stream=stream)
    torch.cuda.synchronize()
    for lps in [int(x) for x in args.levels_per_step.split(",")]:
        eng = default_engine(args.max_active, args.pool_mib, stream=stream, levels_per_step=max(lps, 1),
                             resident=lps == 0)
        if lps == 0 and args.level_lag is not None:
            eng.set_level_lag(args.level_lag)
        native = not args.python_loop
        warm = make_requests(cells, 200, seed=1)
        saturation(eng, cells, warm, native=native)
        reqs = make_requests(cells, args.requests, seed=2)
        sat = saturation(eng, cells, reqs, native=native)
        print(json.dumps({"mode": "saturation", "levels_per_step": lps, **sat}), flush=True)
        rate_sat = sat["served_req_per_s"]
        for load in [float(x) for x in args.loads.split(",")]:
            arr = wl.poisson_arrivals(load * rate_sat, args.requests, seed=424242)
            arr = arr - arr[0]
            res = run_stream(eng, cells, make_requests(cells, args.requests, seed=3), arr, native=native)
            print(json.dumps({"mode": "poisson", "levels_per_step": lps, "load": load, **res}), flush=True)
        # one request per cell per slot (8000 slots/s per cell)
        per_slot = 8000.0 * args.cells
        print(json.dumps({"mode": "note", "levels_per_step": lps,
                          "one_request_per_cell_per_slot_req_per_s": per_slot,
                          "ratio_to_saturation": per_slot / rate_sat}), flush=True)
        eng.close()


if __name__ == "__main__":
    sys.exit(main())
