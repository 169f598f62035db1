"""Build libmfd.so (HIP, gfx950) in-tree with hipcc.

Every device translation unit is compiled with
  -ffp-contract=off   : binary64 arithmetic is a rounded multiply followed by a
                        rounded add wherever the source writes a*b+c (the FP64
                        path is bit-compared with an independent CPU build);
                        binary32 code asks for fused multiply-adds explicitly;
  -Xclang -target-feature -Xclang -packed-fp32-ops : no packed FP32 ops.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmfd.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = [
    "scheme.cpp",
    "mfd_api.cpp",
    "autotune.cpp",
    "batch.cpp",
    "server.cpp",
    "general_api.cpp",
    "kernels_mmfd.hip",
    "kernels_tb.hip",
    "kernels_nse_tb.hip",
    "kernels_lane_tb.hip",
    "kernels_nse3d.hip",
    "kernels_1d_wave.hip",
    "kernels_mesofd_tb.hip",
    "kernels_mesofd.hip",
    "kernels_misc.hip",
    "kernels_batch.hip",
    "kernels_source.hip",
    "kernels_mg.hip",
    "kernels_general.hip",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MFD_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable", "-Wno-unused-but-set-variable"]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _deps_mtime() -> float:
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hdrs.append(os.path.join(HERE, "..", "include", "mfd.h"))
    return max(os.path.getmtime(h) for h in hdrs if os.path.exists(h))


def _compile(src: str, force: bool = True) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if (not force and os.path.exists(obj)
            and os.path.getmtime(obj) > max(os.path.getmtime(path), _deps_mtime())):
        return obj
    cmd = [HIPCC] + COMMON + ["-x", "hip"] + DEVICE + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every source (force=True) or only those changed since their
    object was written, then link libmfd.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), srcs))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, force="--incremental" not in sys.argv)
    sys.exit(0)
