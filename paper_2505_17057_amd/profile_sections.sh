#!/bin/bash
# rocprofv3 kernel-trace statistics of the benchmark's other sections (run from
# the repository root on a machine with the GPU).  Each section runs in a
# profiler process of its own without the headline (bench.py --no-headline),
# and the per-kernel table is split by launch grid, so the kernels of the timed
# plans stand apart from the autotuner's trial plans.  The result databases
# stay in /tmp; only the summaries are written, to
# gpurun_out/profile_<section>.md (copy them into profiles/).
# Usage: profile_sections.sh [section ...]
set -u
R=$(pwd)
O=$R/gpurun_out
mkdir -p "$O"
export TMPDIR=/tmp
for sec in ${@:-c2 variants theta big c1 nse3d source wave burgers batched serving}; do
  echo "profile: $sec"
  CMD="rocprofv3 --kernel-trace --stats -d /tmp/prof_$sec -o p -- python3 bench.py --steps 1 --warmup 0 --no-cpu --no-headline --sections $sec --serve-requests 600"
  (cd /tmp && timeout -k 10 600 rocprofv3 --kernel-trace --stats -d /tmp/prof_$sec -o p -- python3 $R/bench.py --steps 1 --warmup 0 --no-cpu --no-headline --sections $sec --serve-requests 600 > "$O/prof_$sec.txt" 2>&1) || exit 2
  python3 -m paper_2505_17057_amd.profiling stats /tmp/prof_$sec/p_results.db 14 "bench.py section '$sec'" "$CMD" > "$O/profile_$sec.md" || exit 3
  python3 - "$O/prof_$sec.txt" >> "$O/profile_$sec.md" <<'PY'
import json, sys
std = {"metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
       "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"}
for line in open(sys.argv[1]):
    if line.startswith("{"):
        d = json.loads(line)
        print("\nThe section's figures from the same run (under the profiler):\n")
        print("```\n" + json.dumps({k: v for k, v in d.items() if k not in std}, indent=1) + "\n```")
PY
  rm -rf /tmp/prof_$sec
done
