#!/bin/bash
# rocprofv3 counters of one benchmark section's kernels (run from the
# repository root on a machine with the GPU): three counter passes, each a
# profiler process of its own without the headline, then per kernel and
# launch grid the mean of every counter per dispatch, written to
# gpurun_out/counters_<section>.md (copy it into profiles/).
# Usage: profile_counters.sh SECTION KERNEL_NAME_PATTERN
set -u
sec=$1
pat=$2
R=$(pwd)
O=$R/gpurun_out
mkdir -p "$O"
export TMPDIR=/tmp
B="python3 $R/bench.py --steps 1 --warmup 0 --no-cpu --no-headline --sections $sec"
i=0
for pmc in "FETCH_SIZE" "WRITE_SIZE" "SQ_INSTS_VALU SQ_INSTS_LDS SQ_WAVES SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU GRBM_GUI_ACTIVE"; do
  i=$((i + 1))
  echo "counters: $sec pass $i ($pmc)"
  (cd /tmp && timeout -s KILL 300 rocprofv3 --pmc $pmc --kernel-trace -d /tmp/cnt_${sec}_$i -o c -- $B > "$O/cnt_${sec}_$i.txt" 2>&1) || exit 2
done
{
  echo "# rocprofv3 counters: bench.py section '$sec', kernels matching '$pat'"
  echo
  echo "Commands (from the repository root; \`cd /tmp && export TMPDIR=/tmp\` first), one per pass:"
  echo
  echo "    rocprofv3 --pmc FETCH_SIZE --kernel-trace -d /tmp/cnt_1 -o c -- python3 bench.py --steps 1 --warmup 0 --no-cpu --no-headline --sections $sec"
  echo "    rocprofv3 --pmc WRITE_SIZE --kernel-trace -d /tmp/cnt_2 -o c -- (the same)"
  echo "    rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_LDS SQ_WAVES SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU GRBM_GUI_ACTIVE --kernel-trace -d /tmp/cnt_3 -o c -- (the same)"
  echo
  echo "Mean per dispatch (FETCH_SIZE and WRITE_SIZE in KiB, raw: on gfx950 a device copy of B bytes reads B/2 on FETCH_SIZE and B on WRITE_SIZE):"
  echo
  python3 -m paper_2505_17057_amd.profiling counters "$pat" /tmp/cnt_${sec}_1/c_results.db /tmp/cnt_${sec}_2/c_results.db /tmp/cnt_${sec}_3/c_results.db
} > "$O/counters_$sec.md" || exit 3
rm -rf /tmp/cnt_${sec}_1 /tmp/cnt_${sec}_2 /tmp/cnt_${sec}_3
