#!/bin/bash
# rocprofv3 evidence for the headline step kernel (run from the repository
# root on a machine with the GPU; writes raw results under gpurun_out/):
#   1. kernel trace + stats of the headline benchmark,
#   2. FETCH_SIZE and 3. WRITE_SIZE counters, each in a run of its own, with a
#      256 MiB device copy as the counter calibration,
# then summarises them with paper_2505_17057_amd.profiling into gpurun_out/
# (copy the .md and .json into profiles/).
set -u
R=$(pwd)
O=$R/gpurun_out
mkdir -p "$O"
export TMPDIR=/tmp
echo "profile: kernel trace"
(cd /tmp && timeout -k 10 240 rocprofv3 --kernel-trace --stats -d "$O/prof_kt" -o kt -- python3 $R/bench.py --quick --steps 5 --warmup 1 --no-cpu --copy-calibration > "$O/prof_kt.txt" 2>&1) || exit 2
# the counter runs use the plan the autotuner chose in the traced run, and
# the summary takes the kernel that plan runs
read PLAN KNAME KSRC < <(python3 -c "import json,sys
for l in open(sys.argv[1]):
    if l.startswith('{'):
        r = json.loads(l)['roofline']
        print('%d,%d,%d' % (r['time_steps_per_launch'], r['window_rows'], r['window_cols']),
              r['kernel'].split()[0], r['kernel_source'])" "$O/prof_kt.txt")
echo "plan $PLAN kernel $KNAME ($KSRC)"
echo "profile: FETCH_SIZE"
(cd /tmp && timeout -s KILL 240 rocprofv3 --pmc FETCH_SIZE --kernel-trace -d "$O/prof_fetch" -o f -- python3 $R/bench.py --quick --steps 1 --warmup 0 --no-cpu --copy-calibration --plan $PLAN > "$O/prof_fetch.txt" 2>&1) || exit 3
echo "profile: WRITE_SIZE"
(cd /tmp && timeout -s KILL 240 rocprofv3 --pmc WRITE_SIZE --kernel-trace -d "$O/prof_write" -o w -- python3 $R/bench.py --quick --steps 1 --warmup 0 --no-cpu --copy-calibration --plan $PLAN > "$O/prof_write.txt" 2>&1) || exit 4
# the same two counters for the other plans the autotuner picks between runs
ALTS=()
for ALT in 10,106,128 12,112,128 14,116,128 16,120,128; do
  [ "${ALT%%,*}" = "${PLAN%%,*}" ] && continue
  T=${ALT//,/_}
  echo "profile: FETCH_SIZE / WRITE_SIZE at $ALT"
  # (result databases in /tmp: only the summaries come back)
  (cd /tmp && timeout -s KILL 240 rocprofv3 --pmc FETCH_SIZE --kernel-trace -d "/tmp/prof_fetch_$T" -o f -- python3 $R/bench.py --quick --steps 1 --warmup 0 --no-cpu --plan $ALT > "$O/prof_fetch_$T.txt" 2>&1) || exit 5
  (cd /tmp && timeout -s KILL 240 rocprofv3 --pmc WRITE_SIZE --kernel-trace -d "/tmp/prof_write_$T" -o w -- python3 $R/bench.py --quick --steps 1 --warmup 0 --no-cpu --plan $ALT > "$O/prof_write_$T.txt" 2>&1) || exit 5
  ALTS+=(--alt "$ALT:/tmp/prof_fetch_$T/f_results.db:/tmp/prof_write_$T/w_results.db")
  ALTS+=(--command "rocprofv3 --pmc FETCH_SIZE --kernel-trace -d /tmp/prof_fetch_$T -o f -- python3 bench.py --quick --steps 1 --warmup 0 --no-cpu --plan $ALT")
  ALTS+=(--command "rocprofv3 --pmc WRITE_SIZE --kernel-trace -d /tmp/prof_write_$T -o w -- python3 bench.py --quick --steps 1 --warmup 0 --no-cpu --plan $ALT")
done
N=4194304
python3 -m paper_2505_17057_amd.profiling --trace "$O/prof_kt/kt_results.db" \
  --fetch "$O/prof_fetch/f_results.db" --write "$O/prof_write/w_results.db" \
  --kernel "$KNAME" --copy-bytes 268435456 \
  --kernel-source "$KSRC" --bench-log "$O/prof_kt.txt" \
  --algorithmic-bytes-per-step $((8 * N)) --pass-bytes $((8 * N)) \
  --workload "2D linear CDE, D2Q9, 2048x2048, MMFD FP32 (bench.py headline)" \
  --out-md "$O/mmfd_lcde_d2q9_2048_fp32.md" --out-json "$O/traffic_mmfd_lcde_d2q9_2048_fp32.json" \
  --command "rocprofv3 --kernel-trace --stats -d gpurun_out/prof_kt -o kt -- python3 bench.py --quick --steps 5 --warmup 1 --no-cpu --copy-calibration" \
  --command "rocprofv3 --pmc FETCH_SIZE --kernel-trace -d gpurun_out/prof_fetch -o f -- python3 bench.py --quick --steps 1 --warmup 0 --no-cpu --copy-calibration --plan $PLAN" \
  --command "rocprofv3 --pmc WRITE_SIZE --kernel-trace -d gpurun_out/prof_write -o w -- python3 bench.py --quick --steps 1 --warmup 0 --no-cpu --copy-calibration --plan $PLAN" \
  "${ALTS[@]}"
