#!/bin/bash
# rocprofv3 evidence for the headline step kernel (2D NSE, three-level TRT,
# D2Q9, 4096^2, FP32; run from the repository root on a machine with the GPU;
# raw results under gpurun_out/):
#   1. kernel trace + stats of the headline benchmark (autotuned plan),
#   2. FETCH_SIZE, 3. WRITE_SIZE and 4. SQ_INSTS_VALU + SQ_WAVES counters, each
#      in a run of its own on the plan of run 1, with a 256 MiB device copy as
#      the HBM counter calibration,
# then summarises them with paper_2505_17057_amd.profiling into gpurun_out/
# (copy the .md and .json into profiles/).
set -u
R=$(pwd)
O=$R/gpurun_out
mkdir -p "$O"
export TMPDIR=/tmp
B="python3 $R/bench.py --quick --no-cpu --copy-calibration"
echo "profile: kernel trace"
(cd /tmp && timeout -k 10 300 rocprofv3 --kernel-trace --stats -d "$O/prof_kt" -o kt -- $B --steps 2 --warmup 0 > "$O/prof_kt.txt" 2>&1) || exit 2
read PLAN KNAME KSRC < <(python3 -c "import json,sys
for l in open(sys.argv[1]):
    if l.startswith('{'):
        r = json.loads(l)['roofline']
        print('%d,%d,%d' % (r['time_steps_per_launch'], r['window_rows'], r['window_cols']),
              r['kernel'].split()[0], r['kernel_source'])" "$O/prof_kt.txt")
echo "plan $PLAN kernel $KNAME ($KSRC)"
echo "profile: FETCH_SIZE"
(cd /tmp && timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE --kernel-trace -d "$O/prof_fetch" -o f -- $B --steps 1 --warmup 0 --plan $PLAN > "$O/prof_fetch.txt" 2>&1) || exit 3
echo "profile: WRITE_SIZE"
(cd /tmp && timeout -s KILL 300 rocprofv3 --pmc WRITE_SIZE --kernel-trace -d "$O/prof_write" -o w -- $B --steps 1 --warmup 0 --plan $PLAN > "$O/prof_write.txt" 2>&1) || exit 4
echo "profile: SQ_INSTS_VALU SQ_WAVES"
(cd /tmp && timeout -s KILL 300 rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES --kernel-trace -d "$O/prof_valu" -o v -- $B --steps 1 --warmup 0 --plan $PLAN > "$O/prof_valu.txt" 2>&1) || exit 5
N=16777216
C="bench.py --quick --no-cpu --copy-calibration"
python3 -m paper_2505_17057_amd.profiling --trace "$O/prof_kt/kt_results.db" \
  --fetch "$O/prof_fetch/f_results.db" --write "$O/prof_write/w_results.db" \
  --valu "$O/prof_valu/v_results.db" --flops-per-lup 230 --lups-per-step $N \
  --kernel "$KNAME" --copy-bytes 268435456 \
  --kernel-source "$KSRC" --bench-log "$O/prof_kt.txt" \
  --algorithmic-bytes-per-step $((36 * N)) --pass-bytes $((48 * N)) \
  --workload "2D NSE, three-level TRT, D2Q9, 4096x4096, MMFD FP32 (bench.py headline)" \
  --out-md "$O/nse_tb_d2q9_4096_fp32.md" --out-json "$O/counters_nse_tb_d2q9_4096_fp32.json" \
  --command "rocprofv3 --kernel-trace --stats -d gpurun_out/prof_kt -o kt -- python3 $C --steps 2 --warmup 0" \
  --command "rocprofv3 --pmc FETCH_SIZE --kernel-trace -d gpurun_out/prof_fetch -o f -- python3 $C --steps 1 --warmup 0 --plan $PLAN" \
  --command "rocprofv3 --pmc WRITE_SIZE --kernel-trace -d gpurun_out/prof_write -o w -- python3 $C --steps 1 --warmup 0 --plan $PLAN" \
  --command "rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES --kernel-trace -d gpurun_out/prof_valu -o v -- python3 $C --steps 1 --warmup 0 --plan $PLAN"
