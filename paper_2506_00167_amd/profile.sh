#!/bin/bash
# rocprofv3 runs behind the summaries in profiles/. Each pass is its own run:
#  - kernel trace + stats of back-to-back single-codebook builds: the subtree
#    kernel for the E=8 K=3 tree in FP32, BF16 and FP8 and for the E=4 K=2
#    tree in FP32; the level kernel of the 32-cell FP8 stress batch;
#  - HBM traffic: FETCH_SIZE, then WRITE_SIZE, on the same builds and on a
#    plain copy of known size that calibrates both counters;
#  - executed matrix-core operations per format, and matrix-core busy cycles
#    against GPU active cycles.
# Summaries and raw output go to OUT (default prof_out under the repository
# root); the summaries are then copied into profiles/ by hand.
#
#   bash paper_2506_00167_amd/profile.sh [OUT] [PASS ...]
# PASS: trace traffic mfma busy (default: all)
set -o pipefail
ROOT=$(cd "$(dirname "$0")/.." && pwd)
OUT=${1:-$ROOT/prof_out}
shift
PASSES=${*:-trace traffic mfma busy}
mkdir -p "$OUT"
export PYTHONPATH=$ROOT
export TMPDIR=/tmp
cd /tmp || exit 1

build_cmd() {  # workload precision -> the program to profile
    echo "python3 -m paper_2506_00167_amd.profiling build --workload $1 --precision $2 --builds 200"
}
STRESS="python3 -m paper_2506_00167_amd.profiling stress --iters 3"
COPY="python3 -m paper_2506_00167_amd.profiling copy --mib 256 --reps 5"
# (name, workload, precision) of the subtree-kernel runs
RUNS="tree-e8k3:fp32 tree-e8k3:bf16 tree-e8k3:fp8 tiny-e4k2:fp32"

trace() {  # name, command...
    local name=$1; shift
    echo "[prof] trace $name" >&2
    timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d "$OUT/$name" -o run -- "$@" \
        > "$OUT/$name.log" 2>&1 || { echo "[prof] $name failed" >&2; tail -20 "$OUT/$name.log" >&2; return 1; }
}
counter() {  # name, counters, command...
    local name=$1 ctr=$2; shift 2
    echo "[prof] counters $name: $ctr" >&2
    timeout -s KILL 120 rocprofv3 --pmc $ctr --output-format csv -d "$OUT/$name" -o run -- "$@" \
        > "$OUT/$name.log" 2>&1 || { echo "[prof] $name failed" >&2; tail -20 "$OUT/$name.log" >&2; return 1; }
}
summ() {  # out-name dir kernel source-kernel command-string [extra summarize args...]
    local out=$1 dir=$2 kernel=$3 src=$4 cmd=$5; shift 5
    python3 -m paper_2506_00167_amd.profiling summarize "$OUT/$dir" --kernel "$kernel" --source-kernel "$src" \
        --command "$cmd" "$@" > "$OUT/$out.txt"
}
# instantiation prefix of the subtree kernel for a precision
kname() { case $1 in fp32) echo "subtree_kernel<0,";; bf16) echo "subtree_kernel<1,";; fp8) echo "subtree_kernel<2,";; esac; }

for pass in $PASSES; do
case $pass in
trace)
    for r in $RUNS; do
        w=${r%%:*}; p=${r##*:}; cmd=$(build_cmd $w $p)
        trace "trace_${w}_$p" $cmd || exit 1
        summ "subtree_kernel_${w}_${p}_trace" "trace_${w}_$p" "$(kname $p)" subtree \
            "rocprofv3 --kernel-trace --stats --output-format csv -d OUT/trace_${w}_$p -o run -- $cmd" || exit 1
    done
    trace trace_stress $STRESS || exit 1
    summ level_kernel_batch_stress-e16k4_fp8_trace trace_stress level_kernel_batch level \
        "rocprofv3 --kernel-trace --stats --output-format csv -d OUT/trace_stress -o run -- $STRESS" || exit 1
    ;;
traffic)
    counter fetch_copy FETCH_SIZE $COPY && counter write_copy WRITE_SIZE $COPY || exit 1
    for p in fp32 bf16 fp8; do
        cmd=$(build_cmd tree-e8k3 $p)
        counter "fetch_$p" FETCH_SIZE $cmd && counter "write_$p" WRITE_SIZE $cmd || exit 1
        for c in fetch:FETCH_SIZE:fetch_copy write:WRITE_SIZE:write_copy; do
            IFS=: read -r what ctr cdir <<< "$c"
            summ "subtree_kernel_tree-e8k3_${p}_$what" "${what}_$p" "$(kname $p)" subtree \
                "rocprofv3 --pmc $ctr --output-format csv -d OUT/${what}_$p -o run -- $cmd" \
                --copy-dir "$OUT/$cdir" --copy-kernel copyBuffer \
                --command "rocprofv3 --pmc $ctr --output-format csv -d OUT/$cdir -o run -- $COPY" || exit 1
        done
        python3 -m paper_2506_00167_amd.profiling traffic --fetch "$OUT/fetch_$p" --write "$OUT/write_$p" \
            --copy-fetch "$OUT/fetch_copy" --copy-write "$OUT/write_copy" --copy-kernel copyBuffer \
            --kernel "$(kname $p)" --key "subtree/tree-e8k3/$p" --out "$OUT/traffic.json" || exit 1
    done
    counter fetch_stress FETCH_SIZE $STRESS && counter write_stress WRITE_SIZE $STRESS || exit 1
    for c in fetch:FETCH_SIZE:fetch_copy write:WRITE_SIZE:write_copy; do
        IFS=: read -r what ctr cdir <<< "$c"
        summ "level_kernel_batch_stress-e16k4_fp8_$what" "${what}_stress" level_kernel_batch level \
            "rocprofv3 --pmc $ctr --output-format csv -d OUT/${what}_stress -o run -- $STRESS" \
            --copy-dir "$OUT/$cdir" --copy-kernel copyBuffer \
            --command "rocprofv3 --pmc $ctr --output-format csv -d OUT/$cdir -o run -- $COPY" || exit 1
    done
    ;;
mfma)
    # executed matrix-core work in units of 512 operations, per format
    for c in fp32:SQ_INSTS_VALU_MFMA_MOPS_F32 bf16:SQ_INSTS_VALU_MFMA_MOPS_BF16 fp8:SQ_INSTS_VALU_MFMA_MOPS_F8; do
        p=${c%%:*}; ctr=${c##*:}; cmd=$(build_cmd tree-e8k3 $p)
        counter "mops_$p" "$ctr" $cmd || exit 1
        summ "subtree_kernel_tree-e8k3_${p}_mfma_ops" "mops_$p" "$(kname $p)" subtree \
            "rocprofv3 --pmc $ctr --output-format csv -d OUT/mops_$p -o run -- $cmd" || exit 1
    done
    counter mops_stress SQ_INSTS_VALU_MFMA_MOPS_F8 $STRESS || exit 1
    summ level_kernel_batch_stress-e16k4_fp8_mfma_ops mops_stress level_kernel_batch level \
        "rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_F8 --output-format csv -d OUT/mops_stress -o run -- $STRESS" || exit 1
    cmd=$(build_cmd tree-e8k3 fp32)
    counter vfma_fp32 SQ_INSTS_VALU_FMA_F32 $cmd || exit 1
    summ subtree_kernel_tree-e8k3_fp32_valu_fma vfma_fp32 "$(kname fp32)" subtree \
        "rocprofv3 --pmc SQ_INSTS_VALU_FMA_F32 --output-format csv -d OUT/vfma_fp32 -o run -- $cmd" || exit 1
    ;;
busy)
    # matrix-core busy cycles (summed over the SIMDs) against GPU active cycles
    BUSY="SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE"
    for p in fp32 bf16 fp8; do
        cmd=$(build_cmd tree-e8k3 $p)
        counter "busy_$p" "$BUSY" $cmd || exit 1
        summ "subtree_kernel_tree-e8k3_${p}_mfma_busy" "busy_$p" "$(kname $p)" subtree \
            "rocprofv3 --pmc $BUSY --output-format csv -d OUT/busy_$p -o run -- $cmd" || exit 1
    done
    counter busy_stress "$BUSY" $STRESS || exit 1
    summ level_kernel_batch_stress-e16k4_fp8_mfma_busy busy_stress level_kernel_batch level \
        "rocprofv3 --pmc $BUSY --output-format csv -d OUT/busy_stress -o run -- $STRESS" || exit 1
    ;;
*) echo "unknown pass $pass" >&2; exit 2;;
esac
done
echo "[prof] done: $OUT" >&2
