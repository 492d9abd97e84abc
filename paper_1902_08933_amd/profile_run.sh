#!/bin/bash
# Profile the fused step on one workload and write the summaries under profiles/:
#   profiles/fused_step_<workload>_trace.txt  (rocprofv3 --kernel-trace --stats)
#   profiles/fused_step_<workload>_pmc.txt    (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, each
#                                              scaled by the counter's reading for the bandwidth probe)
# Usage (from the repository root): bash paper_1902_08933_amd/profile_run.sh spinodal1024
# Raw rocprofv3 output goes to $RAW_OUT/prof_<workload>/ (default RAW_OUT=prof_raw);
# PROFILE_OUT overrides profiles/.
set -o pipefail
W=${1:-spinodal1024}
RAW=${RAW_OUT:-prof_raw}
if [ "$W" = "sp1024" ]; then
    # single-phase step with a mass source at 1024^2 (incompressible, full force term): kernel
    # trace, then HBM traffic (FETCH_SIZE, WRITE_SIZE, scaled by the same counters on the probe)
    OUT=$RAW/prof_sp1024
    PROF=${PROFILE_OUT:-profiles}
    mkdir -p "$OUT" "$PROF"
    export TMPDIR=/tmp
    CMD="python3 -m paper_1902_08933_amd.profile_step --workload sp1024"
    PROBE="python3 -m paper_1902_08933_amd.profile_step --copy-mib 1024 --steps 2 --probe-blocks 4096"
    echo "profile: kernel trace sp1024" && \
    timeout -k 10 180 rocprofv3 --kernel-trace --stats -d "$OUT/trace" -o run -- $CMD --steps 100 --warmup 10 > "$OUT/trace.log" 2>&1 && \
    echo "profile: FETCH_SIZE sp1024" && \
    timeout -s KILL 90 rocprofv3 --pmc FETCH_SIZE -d "$OUT/fetch" -o run -- $CMD --steps 5 --warmup 1 > "$OUT/fetch.log" 2>&1 && \
    echo "profile: WRITE_SIZE sp1024" && \
    timeout -s KILL 90 rocprofv3 --pmc WRITE_SIZE -d "$OUT/write" -o run -- $CMD --steps 5 --warmup 1 > "$OUT/write.log" 2>&1 && \
    echo "profile: probe FETCH_SIZE" && \
    timeout -s KILL 90 rocprofv3 --pmc FETCH_SIZE -d "$OUT/cfetch" -o run -- $PROBE > "$OUT/cfetch.log" 2>&1 && \
    echo "profile: probe WRITE_SIZE" && \
    timeout -s KILL 90 rocprofv3 --pmc WRITE_SIZE -d "$OUT/cwrite" -o run -- $PROBE > "$OUT/cwrite.log" 2>&1 && \
    python3 -m paper_1902_08933_amd.rocprof_summary --trace "$OUT/trace/run_results.db" --cells 1048576 \
        --kernel sp_step_kernel --alg-bytes-per-cell 92 --sources sp \
        --command "bash paper_1902_08933_amd/profile_run.sh sp1024  (rocprofv3 --kernel-trace --stats -- $CMD --steps 100 --warmup 10)" \
        --out "$PROF/sp_step_sp1024_trace.txt" && \
    python3 -m paper_1902_08933_amd.rocprof_summary --fetch "$OUT/fetch/run_results.db" --write "$OUT/write/run_results.db" \
        --calib-fetch "$OUT/cfetch/run_results.db" --calib-write "$OUT/cwrite/run_results.db" --calib-bytes 1073741824 \
        --cells 1048576 --kernel sp_step_kernel --alg-bytes-per-cell 92 --sources sp \
        --command "bash paper_1902_08933_amd/profile_run.sh sp1024  (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE -- $CMD --steps 5 --warmup 1; calibration: same counters on $PROBE)" \
        --out "$PROF/sp_step_sp1024_pmc.txt"
    exit $?
fi
if [ "$W" = "r4_1024" ]; then
    # single-phase Remark 4 scheme with drag at 1024^2: G pass (100 B/node) and collision (144 B/node)
    OUT=$RAW/prof_r4_1024
    PROF=${PROFILE_OUT:-profiles}
    mkdir -p "$OUT" "$PROF"
    export TMPDIR=/tmp
    CMD="python3 -m paper_1902_08933_amd.profile_step --workload r4_1024 --steps 100 --warmup 10"
    echo "profile: kernel trace r4_1024" && \
    timeout -k 10 180 rocprofv3 --kernel-trace --stats -d "$OUT/trace" -o run -- $CMD > "$OUT/trace.log" 2>&1 && \
    python3 -m paper_1902_08933_amd.rocprof_summary --trace "$OUT/trace/run_results.db" --cells 1048576 \
        --kernel sp_r4_collide_kernel --alg-bytes-per-cell 144 --sources sp \
        --command "bash paper_1902_08933_amd/profile_run.sh r4_1024  (rocprofv3 --kernel-trace --stats -- $CMD)" \
        --out "$PROF/sp_remark4_r4_1024_trace.txt"
    exit $?
fi
if [ "$W" = "d3q15_256" ]; then
    # D3Q15 two-phase step at 256^3: autotuned launch shape, kernel trace, then HBM traffic
    # (FETCH_SIZE, WRITE_SIZE, scaled by the same counters on the copy probe)
    OUT=$RAW/prof_d3q15_256
    PROF=${PROFILE_OUT:-profiles}
    mkdir -p "$OUT" "$PROF"
    export TMPDIR=/tmp
    CELLS=16777216
    SHAPE=$(timeout -k 10 120 python3 -m paper_1902_08933_amd.profile_step --workload d3q15_256 --autotune | tail -1) || exit 1
    echo "profile: autotuned launch shape $SHAPE"
    STEP="python3 -m paper_1902_08933_amd.profile_step --workload d3q15_256 --tile $SHAPE"
    PROBE="python3 -m paper_1902_08933_amd.profile_step --copy-mib 1024 --steps 2 --probe-blocks 4096"
    echo "profile: kernel trace d3q15_256" && \
    timeout -k 10 180 rocprofv3 --kernel-trace --stats -d "$OUT/trace" -o run -- $STEP --steps 50 --warmup 5 > "$OUT/trace.log" 2>&1 && \
    echo "profile: FETCH_SIZE d3q15_256" && \
    timeout -s KILL 90 rocprofv3 --pmc FETCH_SIZE -d "$OUT/fetch" -o run -- $STEP --steps 5 --warmup 1 > "$OUT/fetch.log" 2>&1 && \
    echo "profile: WRITE_SIZE d3q15_256" && \
    timeout -s KILL 90 rocprofv3 --pmc WRITE_SIZE -d "$OUT/write" -o run -- $STEP --steps 5 --warmup 1 > "$OUT/write.log" 2>&1 && \
    echo "profile: probe FETCH_SIZE" && \
    timeout -s KILL 90 rocprofv3 --pmc FETCH_SIZE -d "$OUT/cfetch" -o run -- $PROBE > "$OUT/cfetch.log" 2>&1 && \
    echo "profile: probe WRITE_SIZE" && \
    timeout -s KILL 90 rocprofv3 --pmc WRITE_SIZE -d "$OUT/cwrite" -o run -- $PROBE > "$OUT/cwrite.log" 2>&1 && \
    python3 -m paper_1902_08933_amd.rocprof_summary --trace "$OUT/trace/run_results.db" --cells $CELLS \
        --kernel march3d_kernel --alg-bytes-per-cell 264 --storage-bytes-per-cell 272 --sources d3q15 \
        --command "bash paper_1902_08933_amd/profile_run.sh d3q15_256  (trace: rocprofv3 --kernel-trace --stats -- $STEP --steps 50 --warmup 5)" \
        --out "$PROF/fused_step3d_d3q15_256_trace.txt" && \
    python3 -m paper_1902_08933_amd.rocprof_summary --fetch "$OUT/fetch/run_results.db" --write "$OUT/write/run_results.db" \
        --calib-fetch "$OUT/cfetch/run_results.db" --calib-write "$OUT/cwrite/run_results.db" --calib-bytes 1073741824 \
        --cells $CELLS --kernel march3d_kernel --alg-bytes-per-cell 264 --storage-bytes-per-cell 272 --sources d3q15 \
        --command "bash paper_1902_08933_amd/profile_run.sh d3q15_256  (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE -- $STEP --steps 5 --warmup 1; calibration: same counters on $PROBE)" \
        --out "$PROF/fused_step3d_d3q15_256_pmc.txt"
    exit $?
fi
if [ "$W" = "batch256" ]; then
    # batched persistent step over the 256 seeded instances (the ones frozen after the 200-step
    # warm-up leave the work list; the node count is that of the active ones, and the summaries
    # count only the launches after the warm-up): autotuned strip shape, kernel trace, then HBM
    # traffic (FETCH_SIZE, WRITE_SIZE, scaled by the same counters on the copy probe)
    OUT=$RAW/prof_batch256
    PROF=${PROFILE_OUT:-profiles}
    mkdir -p "$OUT" "$PROF"
    export TMPDIR=/tmp
    LAST=$(timeout -k 10 180 python3 -m paper_1902_08933_amd.profile_step --workload batch256 --autotune | tail -1) || exit 1
    read -r TILE CELLS <<< "$LAST"
    echo "profile: autotuned strip shape $TILE, $CELLS nodes"
    STEP="python3 -m paper_1902_08933_amd.profile_step --workload batch256 --tile $TILE"
    PROBE="python3 -m paper_1902_08933_amd.profile_step --copy-mib 1024 --steps 2 --probe-blocks 4096"
    echo "profile: kernel trace batch256" && \
    timeout -k 10 180 rocprofv3 --kernel-trace --stats -d "$OUT/trace" -o run -- $STEP --steps 40 --warmup 8 > "$OUT/trace.log" 2>&1 && \
    echo "profile: FETCH_SIZE batch256" && \
    timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d "$OUT/fetch" -o run -- $STEP --steps 5 --warmup 1 > "$OUT/fetch.log" 2>&1 && \
    echo "profile: WRITE_SIZE batch256" && \
    timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d "$OUT/write" -o run -- $STEP --steps 5 --warmup 1 > "$OUT/write.log" 2>&1 && \
    echo "profile: probe FETCH_SIZE" && \
    timeout -s KILL 90 rocprofv3 --pmc FETCH_SIZE -d "$OUT/cfetch" -o run -- $PROBE > "$OUT/cfetch.log" 2>&1 && \
    echo "profile: probe WRITE_SIZE" && \
    timeout -s KILL 90 rocprofv3 --pmc WRITE_SIZE -d "$OUT/cwrite" -o run -- $PROBE > "$OUT/cwrite.log" 2>&1 && \
    python3 -m paper_1902_08933_amd.rocprof_summary --trace "$OUT/trace/run_results.db" --cells $CELLS \
        --kernel batch_kernel --alg-bytes-per-cell 160 --storage-bytes-per-cell 168 --sources step --last 40 \
        --command "bash paper_1902_08933_amd/profile_run.sh batch256  (trace: rocprofv3 --kernel-trace --stats -- $STEP --steps 40 --warmup 8; the last 40 launches counted)" \
        --out "$PROF/batch_step_batch256_trace.txt" && \
    python3 -m paper_1902_08933_amd.rocprof_summary --fetch "$OUT/fetch/run_results.db" --write "$OUT/write/run_results.db" \
        --calib-fetch "$OUT/cfetch/run_results.db" --calib-write "$OUT/cwrite/run_results.db" --calib-bytes 1073741824 \
        --cells $CELLS --kernel batch_kernel --alg-bytes-per-cell 160 --storage-bytes-per-cell 168 --sources step --last 5 \
        --command "bash paper_1902_08933_amd/profile_run.sh batch256  (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE -- $STEP --steps 5 --warmup 1, the last 5 launches counted; calibration: same counters on $PROBE)" \
        --out "$PROF/batch_step_batch256_pmc.txt"
    exit $?
fi
if [ "$W" = "bench1024" ] || [ "$W" = "bench4096" ]; then
    # the benchmark's own command (its headline leg only) under the kernel trace: the summary gives
    # the traced average duration of the timed launches of the fused step beside the ms_per_step
    # that the same run's bench.py line reports
    N=${W#bench}
    STEPS=$([ "$N" = "1024" ] && echo 2000 || echo 200)
    OUT=$RAW/prof_$W
    PROF=${PROFILE_OUT:-profiles}
    mkdir -p "$OUT" "$PROF"
    export TMPDIR=/tmp
    CMD="python3 bench.py --workload spinodal$N --steps $STEPS --warmup 20 --no-large --no-im --no-batch --no-surrogate --no-single-phase --no-d3q15 --no-paper-workloads --no-cpu-baseline"
    echo "profile: kernel trace of bench.py on spinodal$N" && \
    timeout -k 10 300 rocprofv3 --kernel-trace --stats -d "$OUT/trace" -o run -- $CMD > "$OUT/trace.log" 2>&1 && \
    python3 -m paper_1902_08933_amd.rocprof_summary --trace "$OUT/trace/run_results.db" --cells $((N * N)) \
        --alg-bytes-per-cell 160 --storage-bytes-per-cell 168 --last $STEPS --bench-log "$OUT/trace.log" \
        --command "bash paper_1902_08933_amd/profile_run.sh $W  (rocprofv3 --kernel-trace --stats -- $CMD; the last $STEPS launches of the fused step, the timed ones, counted)" \
        --out "$PROF/fused_step_bench$N""_trace.txt"
    exit $?
fi
if [ "$W" = "unet1024" ]; then
    # surrogate forward pass at 1024^2 (214 GFLOP): kernel trace of 100 warm-up forwards (the
    # clocks settle) and 10 timed ones; the summary counts the library's kernels of the last 10
    OUT=$RAW/prof_unet1024
    PROF=${PROFILE_OUT:-profiles}
    mkdir -p "$OUT" "$PROF"
    export TMPDIR=/tmp
    CMD="python3 -m paper_1902_08933_amd.profile_unet --h 1024 --w 1024 --warmup 100 --reps 10"
    echo "profile: kernel trace unet1024" && \
    timeout -k 10 180 rocprofv3 --kernel-trace --stats -d "$OUT/trace" -o run -- $CMD > "$OUT/trace.log" 2>&1 && \
    python3 -m paper_1902_08933_amd.rocprof_summary --trace "$OUT/trace/run_results.db" --iterations 10 --sources unet \
        --kernel "lbpf::" --last 10 \
        --flop "$(python3 -m paper_1902_08933_amd.profile_unet --h 1024 --w 1024 --flop-only)" \
        --command "bash paper_1902_08933_amd/profile_run.sh unet1024  (rocprofv3 --kernel-trace --stats -- $CMD)" \
        --out "$PROF/unet_forward_1024_trace.txt"
    exit $?
fi
N=${W#spinodal}
CELLS=$((N * N))
OUT=$RAW/prof_$W
PROF=${PROFILE_OUT:-profiles}
mkdir -p "$OUT" "$PROF"
export TMPDIR=/tmp
# the strip shape the autotuner picks (an unprofiled run), then every profiled run uses it
TILE=$(timeout -k 10 120 python3 -m paper_1902_08933_amd.profile_step --workload $W --autotune | tail -1) || exit 1
echo "profile: autotuned strip shape $TILE"
STEP="python3 -m paper_1902_08933_amd.profile_step --workload $W --tile $TILE"
PROBE="python3 -m paper_1902_08933_amd.profile_step --copy-mib 1024 --steps 2 --probe-blocks 4096"
echo "profile: kernel trace $W" && \
timeout -k 10 180 rocprofv3 --kernel-trace --stats -d "$OUT/trace" -o run -- $STEP --steps 100 --warmup 10 > "$OUT/trace.log" 2>&1 && \
echo "profile: FETCH_SIZE $W" && \
timeout -s KILL 90 rocprofv3 --pmc FETCH_SIZE -d "$OUT/fetch" -o run -- $STEP --steps 5 --warmup 1 > "$OUT/fetch.log" 2>&1 && \
echo "profile: WRITE_SIZE $W" && \
timeout -s KILL 90 rocprofv3 --pmc WRITE_SIZE -d "$OUT/write" -o run -- $STEP --steps 5 --warmup 1 > "$OUT/write.log" 2>&1 && \
echo "profile: probe FETCH_SIZE" && \
timeout -s KILL 90 rocprofv3 --pmc FETCH_SIZE -d "$OUT/cfetch" -o run -- $PROBE > "$OUT/cfetch.log" 2>&1 && \
echo "profile: probe WRITE_SIZE" && \
timeout -s KILL 90 rocprofv3 --pmc WRITE_SIZE -d "$OUT/cwrite" -o run -- $PROBE > "$OUT/cwrite.log" 2>&1 && \
python3 -m paper_1902_08933_amd.rocprof_summary --trace "$OUT/trace/run_results.db" --cells $CELLS \
    --alg-bytes-per-cell 160 --storage-bytes-per-cell 168 --command "bash paper_1902_08933_amd/profile_run.sh $W  (trace: rocprofv3 --kernel-trace --stats -- $STEP --steps 100 --warmup 10)" \
    --out "$PROF/fused_step_${W}_trace.txt" && \
python3 -m paper_1902_08933_amd.rocprof_summary --fetch "$OUT/fetch/run_results.db" --write "$OUT/write/run_results.db" \
    --calib-fetch "$OUT/cfetch/run_results.db" --calib-write "$OUT/cwrite/run_results.db" --calib-bytes 1073741824 \
    --cells $CELLS --alg-bytes-per-cell 160 --storage-bytes-per-cell 168 \
    --command "bash paper_1902_08933_amd/profile_run.sh $W  (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE -- $STEP --steps 5 --warmup 1; calibration: same counters on $PROBE)" \
    --out "$PROF/fused_step_${W}_pmc.txt"
