#!/bin/bash
# rocprofv3 evidence for the 3D NSE step kernel (D3Q19, three-level TRT,
# 512^3, FP32; run from the repository root on a machine with the GPU; raw
# results under gpurun_out/):
#   1. kernel trace + stats of the bench section (100 time steps per solve),
#   2. FETCH_SIZE, 3. WRITE_SIZE, 4. SQ_INSTS_VALU + SQ_WAVES and
#   5. SQ_INSTS_LDS + SQ_LDS_BANK_CONFLICT + SQ_WAIT_INST_LDS + SQ_BUSY_CYCLES,
#      each in a run of its own, with a 256 MiB device copy as the HBM counter
#      calibration,
# then summarises them with paper_2505_17057_amd.profiling into gpurun_out/
# (copy the .md and .json into profiles/).
set -u
R=$(pwd)
O=$R/gpurun_out
mkdir -p "$O"
export TMPDIR=/tmp
B="python3 $R/bench.py --no-headline --no-cpu --copy-calibration --sections nse3d --nse3d-steps 100 --steps 1 --warmup 0"
K="k_nse3d_pp<true, 32, 8, float>"
echo "profile: kernel trace"
(cd /tmp && timeout -k 10 300 rocprofv3 --kernel-trace --stats -d "$O/prof3_kt" -o kt -- $B > "$O/prof3_kt.txt" 2>&1) || exit 2
echo "profile: FETCH_SIZE"
(cd /tmp && timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE --kernel-trace -d "$O/prof3_fetch" -o f -- $B > "$O/prof3_fetch.txt" 2>&1) || exit 3
echo "profile: WRITE_SIZE"
(cd /tmp && timeout -s KILL 300 rocprofv3 --pmc WRITE_SIZE --kernel-trace -d "$O/prof3_write" -o w -- $B > "$O/prof3_write.txt" 2>&1) || exit 4
echo "profile: SQ_INSTS_VALU SQ_WAVES"
(cd /tmp && timeout -s KILL 300 rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES --kernel-trace -d "$O/prof3_valu" -o v -- $B > "$O/prof3_valu.txt" 2>&1) || exit 5
echo "profile: LDS counters"
(cd /tmp && timeout -s KILL 300 rocprofv3 --pmc SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_LDS SQ_BUSY_CYCLES --kernel-trace -d "$O/prof3_lds" -o l -- $B > "$O/prof3_lds.txt" 2>&1) || exit 6
N=134217728
C="bench.py --no-headline --no-cpu --copy-calibration --sections nse3d --nse3d-steps 100 --steps 1 --warmup 0"
python3 -m paper_2505_17057_amd.profiling --trace "$O/prof3_kt/kt_results.db" \
  --fetch "$O/prof3_fetch/f_results.db" --write "$O/prof3_write/w_results.db" \
  --valu "$O/prof3_valu/v_results.db" --more "$O/prof3_lds/l_results.db" \
  --flops-per-lup 560 --lups-per-step $N --plan 1,8,32 \
  --kernel "$K" --copy-bytes 268435456 \
  --kernel-source paper_2505_17057_amd/csrc/kernels_nse3d.hip \
  --algorithmic-bytes-per-step $((48 * N)) --pass-bytes $((48 * N)) \
  --workload "3D NSE, three-level TRT, D3Q19, 512^3, MMFD FP32 (bench.py section nse3d)" \
  --out-md "$O/nse3d_pp_d3q19_512_fp32.md" --out-json "$O/counters_nse3d_pp_d3q19_512_fp32.json" \
  --command "rocprofv3 --kernel-trace --stats -d gpurun_out/prof3_kt -o kt -- python3 $C" \
  --command "rocprofv3 --pmc FETCH_SIZE --kernel-trace -d gpurun_out/prof3_fetch -o f -- python3 $C" \
  --command "rocprofv3 --pmc WRITE_SIZE --kernel-trace -d gpurun_out/prof3_write -o w -- python3 $C" \
  --command "rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES --kernel-trace -d gpurun_out/prof3_valu -o v -- python3 $C" \
  --command "rocprofv3 --pmc SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_LDS SQ_BUSY_CYCLES --kernel-trace -d gpurun_out/prof3_lds -o l -- python3 $C"
