"""Programs to run under rocprofv3, and summaries of what it records.

  python -m paper_2506_00167_amd.profiling build --precision fp32 --builds 50
      C2 codebook builds (device-resident UE state), one launch each.
  python -m paper_2506_00167_amd.profiling stress --iters 5
      the 32-cell FP8 batch.
  python -m paper_2506_00167_amd.profiling copy --mib 256 --reps 5
      a plain device-to-device copy of known size: the calibration of the
      FETCH_SIZE / WRITE_SIZE counters (bytes the counters report per byte the
      copy must move).
  python -m paper_2506_00167_amd.profiling summarize DIR --kernel SUBSTR [--copy-dir DIR --copy-mib N]
      reads rocprofv3 CSV output (kernel_stats / kernel_trace / counter
      collection) and prints a short text summary.
  python -m paper_2506_00167_amd.profiling traffic --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR
         --kernel SUBSTR --key KERNEL/WORKLOAD/PRECISION [--copy-mib N] [--out FILE]
      HBM bytes per launch of the kernel from a FETCH_SIZE run and a
      WRITE_SIZE run, each scaled by what the same counter reports for the
      plain copy of known size; stored in profiles/traffic.json with the hash
      of the kernel sources the counters were taken on.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import sys


def _build(args):
    import torch
    from . import cyrus
    from . import workload as wl
    cfg = wl.WORKLOADS[args.workload].with_precision(args.precision)
    act = None
    if args.precision == "fp8":
        import json
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        act = json.load(open(os.path.join(root, "tests", "golden", "fp8_act_scales.json")))[
            f"{args.workload}/{wl.WEIGHT_SEEDS[args.workload]}"]
    cb = cyrus.Codebook(cfg, wl.make_weights(cfg, wl.WEIGHT_SEEDS[args.workload]), act_scale=act,
                        force_level=args.level)
    ue = cyrus.ue_device_tensor(wl.make_ue_state(cfg.num_ue, wl.ue_seed(0)))
    for _ in range(args.builds):
        cb.build_device(ue)
    torch.cuda.synchronize()
    print(f"{args.builds} builds of {args.workload}/{args.precision} on the {cb.kernel_path} path")


def _stress(args):
    from . import stress
    print(stress.run(args.iters, warmup=1))


def _copy(args):
    import torch
    n = args.mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"{args.reps} copies of {args.mib} MiB")


def _rows(d, pattern):
    out = []
    for p in glob.glob(os.path.join(d, "**", pattern), recursive=True):
        with open(p, newline="") as f:
            out += list(csv.DictReader(f))
    return out


def _counter_per_dispatch(d, kernel, with_duration=False):
    """Average counter values (as recorded) per dispatch of kernels matching
    `kernel`; with_duration: also the mean dispatch duration in ns under the
    counter run (key "duration_ns")."""
    rows = _rows(d, "*counter_collection.csv")
    acc, dur = {}, {}
    for r in rows:
        if kernel not in r.get("Kernel_Name", ""):
            continue
        name = r.get("Counter_Name")
        acc.setdefault(name, {}).setdefault(r.get("Dispatch_Id"), 0.0)
        acc[name][r.get("Dispatch_Id")] += float(r.get("Counter_Value", 0))
        if r.get("End_Timestamp") and r.get("Start_Timestamp"):
            dur[r.get("Dispatch_Id")] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    out = {k: sum(v.values()) / len(v) for k, v in acc.items() if v}
    if with_duration and dur:
        out["duration_ns"] = sum(dur.values()) / len(dur)
    return out


def _summarize(args):
    lines = [f"# rocprofv3 summary: kernels matching '{args.kernel}'", ""]
    for c in args.command or []:
        lines.append(f"command: {c}")
    if args.command:
        lines.append("")
    stats = _rows(args.dir, "*kernel_stats.csv")
    for r in stats:
        if args.kernel in r.get("Name", ""):
            lines.append(f"kernel_stats: name={r['Name'][:120]} calls={r.get('Calls')} "
                         f"avg_ns={r.get('AverageNs')} min_ns={r.get('MinNs')} max_ns={r.get('MaxNs')} "
                         f"total_ns={r.get('TotalDurationNs')}")
    trace = [r for r in _rows(args.dir, "*kernel_trace.csv") if args.kernel in r.get("Kernel_Name", "")]
    if trace:
        durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace]
        durs.sort()
        lines.append(f"kernel_trace: dispatches={len(durs)} avg_us={sum(durs) / len(durs) / 1e3:.2f} "
                     f"p50_us={durs[len(durs) // 2] / 1e3:.2f} max_us={durs[-1] / 1e3:.2f} "
                     f"grid={trace[0].get('Grid_Size_X', trace[0].get('Grid_Size', '?'))} "
                     f"wg={trace[0].get('Workgroup_Size_X', trace[0].get('Workgroup_Size', '?'))} "
                     f"lds={trace[0].get('LDS_Block_Size', trace[0].get('Lds_Size', '?'))} "
                     f"vgpr={trace[0].get('VGPR_Count', '?')} agpr={trace[0].get('Accum_VGPR_Count', '?')} "
                     f"sgpr={trace[0].get('SGPR_Count', '?')} scratch={trace[0].get('Scratch_Size', '?')}")
    pmc = _counter_per_dispatch(args.dir, args.kernel, with_duration=True)
    dur_ns = pmc.pop("duration_ns", None)
    for k, v in sorted(pmc.items()):
        lines.append(f"counter {k}: {v:.1f} per dispatch")
    if dur_ns:
        lines.append(f"dispatch duration under counters: {dur_ns / 1e3:.2f} us average")
    busy = pmc.get("SQ_VALU_MFMA_BUSY_CYCLES")
    if busy and dur_ns:
        # busy cycles are summed over every SIMD of the GPU (4 per CU)
        simds = 4 * args.num_cu
        lines.append(f"mfma_busy_fraction: {busy / (dur_ns * args.clock_ghz * simds):.4f} "
                     f"(SQ_VALU_MFMA_BUSY_CYCLES / (dispatch duration x {args.clock_ghz} GHz x {simds} SIMDs))")
        gui = pmc.get("GRBM_GUI_ACTIVE")
        if gui:
            # GRBM_GUI_ACTIVE is recorded summed over the 8 XCDs (about 8 x
            # 2.4 cycles per ns of dispatch, plus the counter window)
            lines.append(f"mfma_busy_fraction_gui: {busy / (gui / args.xcds * simds):.4f} "
                         f"(SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / {args.xcds} XCDs x {simds} SIMDs))")
    if args.source_kernel:
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        sys.path.insert(0, root)
        from bench import kernel_source_hash
        lines.append(f"source_hash: {kernel_source_hash(args.source_kernel)} (code of the {args.source_kernel} "
                     f"kernel sources this was taken on)")
    if args.copy_dir:
        cp = _counter_per_dispatch(args.copy_dir, args.copy_kernel)
        moved = args.copy_mib * 1024.0  # KiB each way
        for k, v in sorted(cp.items()):
            lines.append(f"copy calibration {k}: {v:.1f} per dispatch for {moved:.0f} KiB moved -> "
                         f"factor {moved / v if v else float('nan'):.4f} KiB per unit")
    print("\n".join(lines))


def _traffic(args):
    import json
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    from bench import kernel_source_hash
    fetch = _counter_per_dispatch(args.fetch, args.kernel).get("FETCH_SIZE")
    write = _counter_per_dispatch(args.write, args.kernel).get("WRITE_SIZE")
    cf = _counter_per_dispatch(args.copy_fetch, args.copy_kernel).get("FETCH_SIZE")
    cw = _counter_per_dispatch(args.copy_write, args.copy_kernel).get("WRITE_SIZE")
    if None in (fetch, write, cf, cw):
        raise SystemExit(f"missing counters: fetch={fetch} write={write} copy_fetch={cf} copy_write={cw}")
    moved_kib = args.copy_mib * 1024.0
    f_factor, w_factor = moved_kib / cf, moved_kib / cw
    entry = {"fetch_kib": fetch * f_factor, "write_kib": write * w_factor,
             "bytes_per_launch": (fetch * f_factor + write * w_factor) * 1024.0,
             "fetch_factor": f_factor, "write_factor": w_factor,
             "raw_fetch_size": fetch, "raw_write_size": write,
             "source_hash": kernel_source_hash(args.key.split("/")[0])}
    path = args.out or os.path.join(root, "profiles", "traffic.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    data[args.key] = entry
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps({args.key: entry}))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("build")
    b.add_argument("--workload", default="tree-e8k3")
    b.add_argument("--precision", default="fp32")
    b.add_argument("--builds", type=int, default=50)
    b.add_argument("--level", action="store_true")
    s = sub.add_parser("stress")
    s.add_argument("--iters", type=int, default=5)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=256)
    c.add_argument("--reps", type=int, default=5)
    m = sub.add_parser("summarize")
    m.add_argument("dir")
    m.add_argument("--kernel", required=True)
    m.add_argument("--copy-dir")
    m.add_argument("--copy-kernel", default="copy")
    m.add_argument("--copy-mib", type=int, default=256)
    m.add_argument("--command", action="append", help="command line that produced DIR (repeatable)")
    m.add_argument("--source-kernel", choices=["subtree", "level"],
                   help="record the hash of this kernel's sources (bench.py trusts a trace only while it matches)")
    m.add_argument("--num-cu", type=int, default=256)
    m.add_argument("--xcds", type=int, default=8)
    m.add_argument("--clock-ghz", type=float, default=2.4)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--key", required=True)
    t.add_argument("--copy-kernel", default="copy")
    t.add_argument("--copy-mib", type=int, default=256)
    t.add_argument("--out", help="traffic file to update (default profiles/traffic.json)")
    args = ap.parse_args(argv)
    {"build": _build, "stress": _stress, "copy": _copy, "summarize": _summarize, "traffic": _traffic}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
