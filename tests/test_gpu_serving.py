"""Continuous-batching engine (many cells, Poisson arrivals) and the batched
stress launch, through the C ABI.

- Host-stepped engine: a request's codebook, alone and in a mix of requests
  of other shapes at other levels, is bit-identical to the same request built
  on its own by one of the two kernels the engine may give it (the
  single-launch subtree kernel for a fresh request on a subtree-capable cell
  under light load, else the level kernel); each of those builds is checked
  against the oracle by the parity tests.
- Resident worker: every request runs the same tile code, so alone, in the
  mix and the cell's own level-path build are all bit-identical; a small cell
  is checked node by node against the BF16 oracle; the worker leaves when
  idle and is relaunched for the next request.
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


def _single_build(cell, ue, weights=None):
    """The one-codebook build the resident worker's result must equal: the
    subtree path where the cell has the shape of the worker's subtree units
    (BF16, two hidden layers of 256), else the level path."""
    cb = cyrus.Codebook(cell.cfg, cell.weights if weights is None else weights)
    cb.build(ue)
    a, _ = cb.export()
    path = cb.kernel_path
    cb.close()
    return a, path


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
        c, ue = reqs[i]
        builds = _own_builds(cells[c], ue)
        for tag, got in (("alone", alone[i]), ("mix", res["results"][i])):
            assert any(np.array_equal(got, b) for b in builds.values()), (
                f"request {i} {tag} equals neither of its cell's own builds ({list(builds)})")
        parity.check_invariants(cells[c].cfg, ue, alone[i])
    eng.close()


def _own_builds(cell, ue):
    """The request built on its own by each kernel the stepped engine may use:
    the cell's own path, and the level kernel."""
    out = {}
    cell.build(ue)
    out[cell.kernel_path] = cell.export()[0]
    if cell.kernel_path != "level":
        lv = cyrus.Codebook(cell.cfg, cell.weights, force_level=True)
        lv.build(ue)
        out["level"] = lv.export()[0]
        lv.close()
    return out


def test_resident_mixed_equals_alone_and_single_build(cells):
    eng = serving.default_engine(max_active=32, pool_mib=128, resident=True)
    reqs = serving.make_requests(cells, 40, seed=11)
    probe_idx = [3, 17, 29]
    alone = {i: _alone(eng, cells[reqs[i][0]], reqs[i][1]) for i in probe_idx}
    arrivals = np.linspace(0.0, 0.002, len(reqs))
    res = serving.run_stream(eng, cells, reqs, arrivals, keep_results=True)
    print(f"[serving] resident mix: {json.dumps({k: v for k, v in res.items() if k != 'results'})}", flush=True)
    assert res["engine"]["completed"] == len(reqs) + len(probe_idx)
    for i in probe_idx:
        c, ue = reqs[i]
        ref, path = _single_build(cells[c], ue)
        assert np.array_equal(alone[i], ref), f"request {i}: resident alone differs from the {path}-path build"
    paths = set()
    for j, (c, ue) in enumerate(reqs):
        ref, path = _single_build(cells[c], ue)
        paths.add(path)
        assert np.array_equal(res["results"][j], ref), f"request {j}: resident mix differs from the {path}-path build"
        parity.check_invariants(cells[c].cfg, ue, ref)
    # both ways of building a request in the worker: subtree units (two
    # hidden layers of 256) and level tiles (512)
    assert paths == {"subtree", "level"}, paths
    eng.close()


def test_resident_matches_same_precision_oracle(cells):
    small = min(range(len(cells)), key=lambda j: cells[j].num_nodes * cells[j].cfg.hidden[0])
    cell = cells[small]
    ue = wl.make_ue_state(cell.cfg.num_ue, 78)
    eng = serving.default_engine(max_active=4, pool_mib=64, resident=True)
    alloc = _alone(eng, cell, ue)
    weights = wl.make_weights(cell.cfg, wl.serving_cell_configs(16, 424242)[small][1])
    ref = cyrus.Codebook(cell.cfg, weights, export_logits=True)
    ref.build(ue)
    ref_alloc, ref_logits = ref.export()
    ref.close()
    assert np.array_equal(ref_alloc, alloc)
    nodes = wl.sample_nodes(cell.cfg, 600, seed=4)
    rep = parity.compare(cell.cfg, weights, ue, ref_alloc, ref_logits, nodes=nodes, precision="bf16", logit_tol=2e-3)
    rep.check(f"resident {cell.cfg}", exact=False)
    eng.close()


def test_resident_memory_admission_and_relaunch(cells):
    import time
    biggest = max(c.num_nodes * c.cfg.num_ue for c in cells)
    pool = 3 * biggest + (1 << 20)  # the worker's tables plus a few state arrays
    eng = cyrus.Engine(pool, 3 * biggest + (2 << 20), max_active=16, resident=True)
    reqs = serving.make_requests(cells, 24, seed=12)
    res = serving.run_stream(eng, cells, reqs, np.zeros(len(reqs)), keep_results=True)
    st = res["engine"]
    print(f"[serving] resident small pool: {st}", flush=True)
    assert st["completed"] == 24 and st["deferred_memory"] > 0
    assert st["pool_bytes_peak"] <= pool
    launches = st["steps"]
    time.sleep(0.2)  # the worker leaves after about 40 ms idle
    c, ue = reqs[0]
    again = _alone(eng, cells[c], ue)
    assert eng.stats()["steps"] == launches + 1, "the idle worker was not relaunched"
    assert np.array_equal(again, res["results"][0])
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


@pytest.mark.parametrize("resident", [False, True])
@pytest.mark.parametrize("native", [True, False])
def test_poisson_stream_short(cells, resident, native):
    # the library's own request loop (cyrus_engine_run) and the Python loop
    # over submit / step / completed / result serve the same stream; every
    # request completes, and with the resident worker both loops return the
    # same codebooks
    eng = serving.default_engine(max_active=64, pool_mib=256, resident=resident)
    reqs = serving.make_requests(cells, 300, seed=14)
    arr = wl.poisson_arrivals(20000.0, len(reqs))
    arr = arr - arr[0]
    res = serving.run_stream(eng, cells, reqs, arr, keep_results=resident, native=native)
    print(f"[serving] poisson 20k req/s, resident={resident}, native={native}: "
          f"{json.dumps({k: v for k, v in res.items() if k != 'results'})}", flush=True)
    assert res["engine"]["completed"] == 300 and res["engine"]["submitted"] == 300
    assert res["request_loop"] == ("native" if native else "python")
    assert res["latency_us"]["p50"] > 0
    if resident:
        for i in (0, 150, 299):
            c, ue = reqs[i]
            assert np.array_equal(res["results"][i], _single_build(cells[c], ue)[0]), f"request {i}"
    eng.close()


def test_resident_tile_order_does_not_change_results(cells):
    # first come, first served (lag 0) and a lag far beyond the stream: the
    # same codebooks as the single builds, and out-of-range lags are refused
    for lag in (0, 4096):
        eng = serving.default_engine(max_active=64, pool_mib=256, resident=True).set_level_lag(lag)
        reqs = serving.make_requests(cells, 120, seed=18)
        arr = wl.poisson_arrivals(20000.0, len(reqs), seed=19)
        res = serving.run_stream(eng, cells, reqs, arr - arr[0], keep_results=True)
        assert res["engine"]["completed"] == 120
        for i in (0, 41, 119):
            c, ue = reqs[i]
            assert np.array_equal(res["results"][i], _single_build(cells[c], ue)[0]), f"lag {lag}, request {i}"
        with pytest.raises(cyrus.CyrusError) as ei:
            eng.set_level_lag(-1)
        assert ei.value.status == -2
        eng.close()


def test_native_loop_refuses_bad_arrivals(cells):
    eng = serving.default_engine(max_active=4, pool_mib=64)
    reqs = serving.make_requests(cells, 3, seed=15)
    with pytest.raises(cyrus.CyrusError) as ei:
        eng.run([cells[c] for c, _ in reqs], [u for _, u in reqs], [0.0, 10.0, 5.0])
    assert ei.value.status == -2
    assert eng.stats()["submitted"] == 0  # refused before any submit
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


def test_resident_relaunch_after_record_table_keeps_full_width(cells):
    # A worker launch admits at most 2,048 requests; the next request makes
    # it stop admitting and leave, and the host relaunches it. Its tile
    # workgroups must stay until every admitted request has finished: had they
    # left at once, the later levels of the requests in flight (hundreds of
    # tiles for the 512-wide K = 4 cells) would fall to the few workgroups
    # still at work, and the requests queued behind them would wait tens of
    # milliseconds.
    eng = serving.default_engine(max_active=128, pool_mib=256, resident=True)
    reqs = serving.make_requests(cells, 2300, seed=16)
    arr = wl.poisson_arrivals(12000.0, len(reqs), seed=17)
    res = serving.run_stream(eng, cells, reqs, arr - arr[0])
    print(f"[serving] 2300 requests at 12k req/s: {json.dumps(res)}", flush=True)
    assert res["engine"]["completed"] == 2300
    assert res["engine"]["steps"] >= 2  # the record table ran out at least once
    # the stall delayed every request queued behind the narrowed launch (p99
    # in the tens of milliseconds); a single slow request is another matter
    assert res["latency_us"]["p99"] < 5000.0, res["latency_us"]
    eng.close()


def test_batch_completion_event_covers_every_codebook():
    # A device batch completes all its codebooks with one event carried by
    # its last launch: export (which waits for the handle's last build)
    # right after the enqueue, with no device synchronization, must see each
    # whole codebook; a later single build of one handle waits on its own
    # event again, and a host-state batch after it re-uses the staging area.
    import torch
    from paper_2506_00167_amd import stress
    cfg, cells_, ues = stress.make_cells(n=8)
    cyrus.build_batch_device(cells_, ues)
    torch.cuda.synchronize()
    ref = [c.export()[0] for c in cells_]
    for rep in range(3):
        cyrus.build_batch_device(cells_, ues)
        for j, c in enumerate(cells_):  # no synchronize: export waits for the batch's event
            assert np.array_equal(c.export()[0], ref[j]), f"repeat {rep}, cell {j}"
    cells_[3].build_device(ues[3])
    assert np.array_equal(cells_[3].export()[0], ref[3])
    host_ues = [wl.make_ue_state(cfg.num_ue, 5_000_000 + j) for j in range(8)]
    for rep in range(2):
        cyrus.build_batch(cells_, host_ues)
        for j, c in enumerate(cells_):
            c.wait()
            assert np.array_equal(c.export()[0], ref[j]), f"host batch {rep}, cell {j}"
    for c in cells_:
        c.close()


def test_oversize_request_is_refused(cells):
    """A request whose tree can never fit the pools is refused at submit, so
    it cannot block the FIFO; later requests still complete."""
    from paper_2506_00167_amd import stress
    cfg, big, _ = stress.make_cells(n=1, precision="bf16")
    eng = cyrus.Engine(2 << 20, 4 << 20, max_active=8)  # the slots and a few small trees
    with pytest.raises(cyrus.CyrusError) as ei:
        eng.submit(big[0], wl.make_ue_state(cfg.num_ue, 1))
    assert ei.value.status == -3
    small = min(cells, key=lambda c: c.num_nodes * c.cfg.num_ue)
    ue = wl.make_ue_state(small.cfg.num_ue, 2)
    alloc = _alone(eng, small, ue)
    parity.check_invariants(small.cfg, ue, alloc)
    eng.close()
    big[0].close()


def test_resident_weight_refresh_reuses_buffers(cells):
    """Weight refreshes while the resident worker stays up: the codebook
    handle double-buffers its weights, so the second refresh overwrites the
    buffer the first request read. Every request must see the weights current
    at its admission (the worker drops its cached lines when the host reports a
    refresh), a refresh is refused while an admitted request holds the buffer
    it would overwrite, and results equal fresh single-codebook builds."""
    small = min(range(len(cells)), key=lambda j: cells[j].num_nodes * cells[j].cfg.hidden[0])
    cell = cells[small]
    cfg = cell.cfg
    w1 = cell.weights
    w2 = wl.make_weights(cfg, 9001)
    w3 = wl.make_weights(cfg, 9002)
    ue = wl.make_ue_state(cfg.num_ue, 31)

    def fresh(weights):
        return _single_build(cell, ue, weights)[0]

    refs = [fresh(w) for w in (w1, w2, w3)]
    assert not np.array_equal(refs[0], refs[1]) and not np.array_equal(refs[1], refs[2])
    eng = serving.default_engine(max_active=8, pool_mib=64, resident=True)
    try:
        got = [_alone(eng, cell, ue)]
        cell.set_weights(w2)
        got.append(_alone(eng, cell, ue))
        cell.set_weights(w3)  # back into the first buffer
        got.append(_alone(eng, cell, ue))
        for k in range(3):
            assert np.array_equal(got[k], refs[k]), f"request after refresh {k}: not the current weights' codebook"
        # an admitted request keeps its buffer: the refresh that would overwrite it waits
        t = eng.submit(cell, ue)
        eng.step()
        with pytest.raises(cyrus.CyrusError) as ei:
            cell.set_weights(w1)  # would overwrite w2's buffer, held by no one: allowed
            cell.set_weights(w2)  # would overwrite w3's buffer, held by the request
        assert ei.value.status == -5
        while True:
            eng.step()
            done = dict(eng.completed())
            if t in done:
                break
        assert np.array_equal(eng.result(t), refs[2]), "the admitted request did not keep its weights"
    finally:
        eng.close()
        cell.set_weights(w1)
