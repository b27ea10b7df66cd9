#!/bin/bash
# rocprofv3 runs behind the summaries in profiles/. Each pass is its own run:
# kernel trace + stats of bench.py (the FP32 subtree kernel, C2) and of the
# 32-cell FP8 stress batch (level kernel), then one counter per run
# (FETCH_SIZE, WRITE_SIZE) on single-codebook builds and on a plain copy of
# known size that calibrates the counters, then the subtree kernel's executed
# matrix-core and vector FMA operations. Summaries and raw output go to OUT
# (default prof_out under the repository root).
#
#   bash paper_2506_00167_amd/profile.sh [OUT]
set -o pipefail
ROOT=$(cd "$(dirname "$0")/.." && pwd)
OUT=${1:-$ROOT/prof_out}
mkdir -p "$OUT"
export PYTHONPATH=$ROOT
export TMPDIR=/tmp
cd /tmp || exit 1

BENCH="python3 $ROOT/bench.py --steps 300 --warmup 30 --latency-builds 100 --no-cpu --no-critic --legs fp32 --context-legs="
BUILD="python3 -m paper_2506_00167_amd.profiling build --workload tree-e8k3 --precision fp32 --builds 50"
STRESS="python3 -m paper_2506_00167_amd.profiling stress --iters 3"
COPY="python3 -m paper_2506_00167_amd.profiling copy --mib 256 --reps 5"

trace() {  # name, command...
    local name=$1; shift
    echo "[prof] $name" >&2
    timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d "$OUT/$name" -o run -- "$@" \
        > "$OUT/$name.log" 2>&1 || { echo "[prof] $name failed" >&2; tail -20 "$OUT/$name.log" >&2; return 1; }
}
counter() {  # name, counter, command...
    local name=$1 ctr=$2; shift 2
    echo "[prof] $name" >&2
    timeout -s KILL 120 rocprofv3 --pmc "$ctr" --output-format csv -d "$OUT/$name" -o run -- "$@" \
        > "$OUT/$name.log" 2>&1 || { echo "[prof] $name failed" >&2; tail -20 "$OUT/$name.log" >&2; return 1; }
}
summ() {  # out-name, dir, kernel, command-string
    python3 -m paper_2506_00167_amd.profiling summarize "$OUT/$2" --kernel "$3" --command "$4" > "$OUT/$1.txt"
}

trace trace_bench $BENCH &&
trace trace_stress $STRESS &&
counter fetch_subtree FETCH_SIZE $BUILD &&
counter write_subtree WRITE_SIZE $BUILD &&
counter fetch_copy FETCH_SIZE $COPY &&
counter write_copy WRITE_SIZE $COPY &&
counter fetch_stress FETCH_SIZE $STRESS &&
counter write_stress WRITE_SIZE $STRESS || exit 1

P="rocprofv3 --kernel-trace --stats --output-format csv -d OUT/trace_bench -o run -- $BENCH"
summ subtree_kernel_tree-e8k3_fp32_trace trace_bench subtree_kernel "$P" &&
summ level_kernel_batch_stress-e16k4_fp8_trace trace_stress level_kernel_batch \
    "rocprofv3 --kernel-trace --stats --output-format csv -d OUT/trace_stress -o run -- $STRESS" &&
python3 -m paper_2506_00167_amd.profiling summarize "$OUT/fetch_subtree" --kernel subtree_kernel \
    --copy-dir "$OUT/fetch_copy" --copy-kernel copyBuffer \
    --command "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch_subtree -o run -- $BUILD" \
    --command "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch_copy -o run -- $COPY" \
    > "$OUT/subtree_kernel_tree-e8k3_fp32_fetch.txt" &&
python3 -m paper_2506_00167_amd.profiling summarize "$OUT/write_subtree" --kernel subtree_kernel \
    --copy-dir "$OUT/write_copy" --copy-kernel copyBuffer \
    --command "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write_subtree -o run -- $BUILD" \
    --command "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write_copy -o run -- $COPY" \
    > "$OUT/subtree_kernel_tree-e8k3_fp32_write.txt" &&
python3 -m paper_2506_00167_amd.profiling summarize "$OUT/fetch_stress" --kernel level_kernel_batch \
    --copy-dir "$OUT/fetch_copy" --copy-kernel copyBuffer \
    --command "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch_stress -o run -- $STRESS" \
    > "$OUT/level_kernel_batch_stress-e16k4_fp8_fetch.txt" &&
python3 -m paper_2506_00167_amd.profiling summarize "$OUT/write_stress" --kernel level_kernel_batch \
    --copy-dir "$OUT/write_copy" --copy-kernel copyBuffer \
    --command "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write_stress -o run -- $STRESS" \
    > "$OUT/level_kernel_batch_stress-e16k4_fp8_write.txt" &&
python3 -m paper_2506_00167_amd.profiling traffic --fetch "$OUT/fetch_subtree" --write "$OUT/write_subtree" \
    --copy-fetch "$OUT/fetch_copy" --copy-write "$OUT/write_copy" --copy-kernel copyBuffer \
    --kernel subtree_kernel --key subtree/tree-e8k3/fp32 --out "$OUT/traffic.json" || exit 1

# work the FP32 subtree kernel executes: FP32 matrix-core operations (in units
# of 512) and vector FMA instructions (one per wave), to set beside the
# algorithmic FLOP count of a build
counter mfma_subtree SQ_INSTS_VALU_MFMA_MOPS_F32 $BUILD &&
counter vfma_subtree SQ_INSTS_VALU_FMA_F32 $BUILD &&
python3 -m paper_2506_00167_amd.profiling summarize "$OUT/mfma_subtree" --kernel subtree_kernel \
    --command "rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_F32 --output-format csv -d OUT/mfma_subtree -o run -- $BUILD" \
    > "$OUT/subtree_kernel_tree-e8k3_fp32_mfma_ops.txt" &&
python3 -m paper_2506_00167_amd.profiling summarize "$OUT/vfma_subtree" --kernel subtree_kernel \
    --command "rocprofv3 --pmc SQ_INSTS_VALU_FMA_F32 --output-format csv -d OUT/vfma_subtree -o run -- $BUILD" \
    > "$OUT/subtree_kernel_tree-e8k3_fp32_valu_fma.txt" &&
echo "[prof] done: $OUT" >&2
