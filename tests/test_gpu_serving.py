"""Continuous-batching engine (many cells, Poisson arrivals) and the batched
stress launch, through the C ABI.

- A request's codebook is bit-identical alone and in a mix of requests of
  other shapes at other levels, and equal to the same cell's own level-path
  build (the engine uses the same kernel).
- Memory admission: with a pool that holds only a few trees, every request
  still completes, admissions are deferred, and the pool high-water mark stays
  within the pool.
- The 32-cell FP8 stress batch matches each cell's single build bit for bit
  and the same-precision oracle on sampled nodes.
"""
import json
import os

import numpy as np
import pytest

from paper_2506_00167_amd import cyrus
from paper_2506_00167_amd import serving
from paper_2506_00167_amd import workload as wl
from tests import parity

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cells():
    import torch
    cs = serving.make_cells(16, seed=424242)
    torch.cuda.synchronize()
    yield cs
    for c in cs:
        c.close()


def _alone(engine, cell, ue):
    t = engine.submit(cell, ue)
    while True:
        engine.step()
        done = dict(engine.completed())
        if t in done:
            return engine.result(t)


@pytest.mark.parametrize("levels_per_step", [1, 7])
def test_mixed_equals_alone_and_single_build(cells, levels_per_step):
    eng = serving.default_engine(max_active=32, pool_mib=128, levels_per_step=levels_per_step)
    reqs = serving.make_requests(cells, 40, seed=11)
    probe_idx = [3, 17, 29]
    alone = {i: _alone(eng, cells[reqs[i][0]], reqs[i][1]) for i in probe_idx}
    # the mix: all 40 submitted at staggered times so they overlap at different levels
    arrivals = np.linspace(0.0, 0.002, len(reqs))
    res = serving.run_stream(eng, cells, reqs, arrivals, keep_results=True)
    print(f"[serving] mix: {json.dumps({k: v for k, v in res.items() if k != 'results'})}", flush=True)
    assert res["engine"]["steps"] > 0
    for i in probe_idx:
        assert np.array_equal(res["results"][i], alone[i]), f"request {i} differs alone vs in the mix"
        c, ue = reqs[i]
        cells[c].build(ue)
        single, _ = cells[c].export()
        assert np.array_equal(single, alone[i]), f"request {i} differs from the cell's own build"
        parity.check_invariants(cells[c].cfg, ue, alone[i])
    eng.close()


def test_engine_matches_same_precision_oracle(cells):
    # a small cell of the mix, checked node by node against the BF16 oracle
    small = min(range(len(cells)), key=lambda j: cells[j].num_nodes * cells[j].cfg.hidden[0])
    cell = cells[small]
    ue = wl.make_ue_state(cell.cfg.num_ue, 77)
    eng = serving.default_engine(max_active=4, pool_mib=64)
    alloc = _alone(eng, cell, ue)
    weights = wl.make_weights(cell.cfg, wl.serving_cell_configs(16, 424242)[small][1])
    # the engine keeps no logits: the same cell built on its own by the same
    # kernel, with logits exported, must give the engine's codebook bit for
    # bit, and carries the per-node logit error into the oracle gate
    ref = cyrus.Codebook(cell.cfg, weights, export_logits=True)
    assert ref.kernel_path == cell.kernel_path
    ref.build(ue)
    ref_alloc, ref_logits = ref.export()
    ref.close()
    assert np.array_equal(ref_alloc, alloc)
    nodes = wl.sample_nodes(cell.cfg, 600, seed=3)
    rep = parity.compare(cell.cfg, weights, ue, ref_alloc, ref_logits, nodes=nodes, precision="bf16", logit_tol=2e-3)
    print(f"[serving] oracle sample {cell.cfg}: {rep.as_dict()}", flush=True)
    rep.check(f"serving {cell.cfg}", exact=False)
    eng.close()


def test_memory_admission_defers_and_completes(cells):
    biggest = max(c.num_nodes * c.cfg.num_ue for c in cells)
    pool = 4 * 2 * biggest + (2 << 20)  # descriptor slots plus a few trees
    eng = cyrus.Engine(pool, pool + (4 << 20), max_active=16)
    reqs = serving.make_requests(cells, 24, seed=12)
    res = serving.run_stream(eng, cells, reqs, np.zeros(len(reqs)))
    st = res["engine"]
    print(f"[serving] small pool: {st}", flush=True)
    assert st["completed"] == 24
    assert st["deferred_memory"] > 0
    assert st["pool_bytes_peak"] <= pool
    assert st["pool_bytes_used"] < pool
    eng.close()


def test_batch_slot_admission(cells):
    eng = serving.default_engine(max_active=2, pool_mib=128)
    reqs = serving.make_requests(cells, 10, seed=13)
    res = serving.run_stream(eng, cells, reqs, np.zeros(len(reqs)))
    assert res["engine"]["completed"] == 10 and res["engine"]["deferred_batch"] > 0
    eng.close()


def test_poisson_stream_short(cells):
    eng = serving.default_engine(max_active=64, pool_mib=256)
    reqs = serving.make_requests(cells, 300, seed=14)
    arr = wl.poisson_arrivals(20000.0, len(reqs))
    arr = arr - arr[0]
    res = serving.run_stream(eng, cells, reqs, arr)
    print(f"[serving] poisson 20k req/s: {json.dumps(res)}", flush=True)
    assert res["engine"]["completed"] == 300
    assert res["latency_us"]["p50"] > 0
    eng.close()


def test_stress_batch_equals_single_and_oracle():
    import torch
    from paper_2506_00167_amd import stress
    cfg, cells_, ues = stress.make_cells(n=8, export_logits=True)
    cyrus.build_batch_device(cells_, ues)
    torch.cuda.synchronize()
    exported = [c.export() for c in cells_]
    batch = [a for a, _ in exported]
    scales = json.load(open(os.path.join(ROOT, "tests", "golden", "fp8_act_scales.json")))
    base = wl.WEIGHT_SEEDS["stress-e16k4"]
    for j in (0, 5):
        c = cells_[j]
        c.build_device(ues[j])
        torch.cuda.synchronize()
        single, _ = c.export()
        assert np.array_equal(single, batch[j])
        ue = wl.make_ue_state(cfg.num_ue, 5_000_000 + j)
        parity.check_invariants(cfg, ue, batch[j])
        nodes = wl.sample_nodes(cfg, 150, seed=20 + j)
        rep = parity.compare(cfg, wl.make_weights(cfg, base + j), ue, batch[j], exported[j][1], nodes=nodes,
                             precision="fp8", act_scale=scales[f"stress-e16k4/{base + j}"], logit_tol=5e-2)
        print(f"[stress] cell {j}: {rep.as_dict()}", flush=True)
        assert rep.cond_unexplained == 0
    for c in cells_:
        c.close()
