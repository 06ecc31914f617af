#!/bin/bash
# Profiles of the benchmark workload (run from the repository root on the GPU machine).
#   1. kernel trace + per-kernel statistics of a short benchmark run
#   2. HBM byte counters (FETCH_SIZE, then WRITE_SIZE) of the same run
#   3. the same counters for a plain 1 GiB copy, to scale them
# Raw output goes to gpurun_out/; the summaries kept in profiles/ quote it.
set -o pipefail
cd /tmp && export TMPDIR=/tmp && cd "$GRAFT_REPO_ROOT" || exit 1
OUT=gpurun_out/prof
mkdir -p $OUT
echo "[prof] kernel trace"
timeout -k 10 400 rocprofv3 --kernel-trace --stats -d $OUT/trace -o bench -- \
  python3 bench.py --steps 10 --warmup 2 --no-cpu-baseline --fit-evals 0 > $OUT/trace_bench.json 2> $OUT/trace_bench.err || exit $?
echo "[prof] FETCH_SIZE"
timeout -s KILL 400 rocprofv3 --pmc FETCH_SIZE -d $OUT/fetch -o bench -- \
  python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --fit-evals 0 > $OUT/fetch_bench.json 2> $OUT/fetch_bench.err || exit $?
echo "[prof] WRITE_SIZE"
timeout -s KILL 400 rocprofv3 --pmc WRITE_SIZE -d $OUT/write -o bench -- \
  python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --fit-evals 0 > $OUT/write_bench.json 2> $OUT/write_bench.err || exit $?
echo "[prof] copy calibration"
timeout -s KILL 200 rocprofv3 --pmc FETCH_SIZE -d $OUT/copy_fetch -o copy -- python3 bench.py --copy-calibration > $OUT/copy1.json 2>&1 || exit $?
timeout -s KILL 200 rocprofv3 --pmc WRITE_SIZE -d $OUT/copy_write -o copy -- python3 bench.py --copy-calibration > $OUT/copy2.json 2>&1 || exit $?
echo "[prof] done"
find $OUT -name "*.csv" | head -50
