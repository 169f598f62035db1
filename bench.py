"""Benchmark of the MesoFD / MMFD time step on one MI355X.

Workload (the one the headline metric is quoted on): 2D anisotropic linear
CDE, D2Q9, periodic 2048 x 2048, K = [[0.02,0.005],[0.005,0.01]],
u = (0.05, 0.03), dt = 2^-18, SRT coefficients, Gaussian hill + seeded noise,
10 000 time steps per solve.  One benchmark "step" is one full solve
(10 000 time steps of the MMFD form in FP32 plus an FP64 mass reduction);
the other forms/precisions of the same workload and an HBM-resident 8192^2
point are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
TIME_STEPS = 10000
N_SIDE = 2048


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--quick", action="store_true", help="headline only (for profiling)")
    return p.parse_args()


def c2_solver(M, cfg, precision, form, torch_stream):
    s = M.Solver("D2Q9", cfg["n"], cfg["dx"], precision, form)
    s.set_equation("lcde", u=cfg["u"], K=cfg["K"], lambda_bar=cfg["lambda_bar"])
    a, ah = M.mfd_preset("srt")
    s.set_scheme("two_level", a, dt=cfg["dt"])
    s.set_stream(torch_stream.cuda_stream)
    s.set_state(cfg["phi0"].astype(s.dtype))
    return s


def timed_steps(torch, s, nsteps, reps=1, reduce_each=True):
    """Wall time (ms) of `reps` x `nsteps` time steps on the solver's stream,
    bracketed by events and synchronisation on both sides."""
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        s.step(nsteps)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    if reduce_each:
        s.reduce()
    return ms


def launch_durations(torch, s, tb, n=200):
    """Mean GPU duration of one launch of the step kernel: events recorded on
    the solver's stream around each of n calls that advance `tb` steps (one
    blocked launch, or one single-step launch when tb = 1)."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record()
        s.step(tb)
        b.record()
    torch.cuda.synchronize()
    d = [a.elapsed_time(b) for a, b in evs]
    return float(np.mean(d)), float(np.median(d))


def stored_traffic(kernel_src):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_mmfd_lcde_d2q9_2048_fp32.json")
    if not os.path.exists(path):
        return None, None
    info = json.load(open(path))
    sha = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if info.get("kernel_source_sha256") != sha:
        return None, info
    return info.get("hbm_bytes_per_launch"), info


def cpu_baseline(cfg, budget_s=15.0):
    """The FP64 oracle (MMFD form) on the host cores, bounded sample."""
    from oracle import native as O
    from oracle import scheme as S

    spec = dict(lattice="D2Q9", n=cfg["n"], dx=cfg["dx"], dt=cfg["dt"], u=cfg["u"], K=cfg["K"],
                lambda_bar=1, a=S.preset_srt()[0])
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    spec["nthreads"] = threads
    phi = cfg["phi0"].copy()
    N = phi.size
    t0 = time.perf_counter()
    steps = 0
    while True:
        phi = O.mmfd_step(spec, phi)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= 2000:
            break
    return dict(value=N * steps / el / 1e9, unit="GLUPS", cores=threads, kind="oracle",
                sample="%d MMFD FP64 time steps of the 2048^2 D2Q9 LCDE workload (%.1f s)" % (steps, el))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2505_17057_amd import mfd as M
    import mfd_inputs as I

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    cfg = I.c2_hill_2d(n=N_SIDE)
    N = N_SIDE * N_SIDE

    # ---------------------------------------------------------- headline
    s32 = c2_solver(M, cfg, "fp32", "mmfd", stream)
    tb = s32.autotune()
    for _ in range(args.warmup):
        timed_steps(torch, s32, TIME_STEPS)
    total_ms = 0.0
    for _ in range(args.steps):
        total_ms += timed_steps(torch, s32, TIME_STEPS)
    ms_per_step = total_ms / args.steps
    glups = N * TIME_STEPS / (ms_per_step * 1e-3) / 1e9

    # dominant kernel: one launch advances `tb` time steps of N nodes
    mean_ms, med_ms = launch_durations(torch, s32, tb, 200)
    alg_bytes = 8.0 * N * tb  # read phi^n, write phi^(n+1): 8 B per LUP in FP32
    achieved = alg_bytes / (mean_ms * 1e-3) / 1e9
    kernel_src = os.path.join(ROOT, "paper_2505_17057_amd", "csrc", "kernels_tb.hip" if tb > 1 else "kernels_mmfd.hip")
    traffic, tinfo = stored_traffic(kernel_src)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel=("mmfd_tb" if tb > 1 else "mmfd_plane") + " D2Q9 LCDE FP32",
                    launch_ms_mean=round(mean_ms, 5), launch_ms_median=round(med_ms, 5),
                    time_steps_per_launch=tb, algorithmic_bytes_per_launch=alg_bytes)

    extra = {}
    if not args.quick:
        # ------------------------------------------------------ variants
        variants = {}
        finals = {}
        for prec, form, nsteps in (("fp64", "mmfd", TIME_STEPS), ("fp32", "mesofd", TIME_STEPS),
                                   ("fp64", "mesofd", TIME_STEPS)):
            sv = c2_solver(M, cfg, prec, form, stream)
            sv.autotune()
            ms = timed_steps(torch, sv, nsteps, reduce_each=False)
            bpl = {("fp64", "mmfd"): 16, ("fp32", "mesofd"): 72, ("fp64", "mesofd"): 144}[(prec, form)]
            g = N * nsteps / (ms * 1e-3) / 1e9
            variants["%s_%s" % (form, prec)] = dict(glups=round(g, 2), alg_gbs=round(g * bpl, 1),
                                                    frac_hbm=round(g * bpl / HBM_PEAK_GBS, 4),
                                                    bytes_per_lup=bpl, ms_per_solve=round(ms, 3))
            finals[(prec, form)] = sv.get_state().astype(np.float64)
            sv.close()
        # FP32 error of the full 10 000-step run against the FP64 run
        s32b = c2_solver(M, cfg, "fp32", "mmfd", stream)
        s32b.step(TIME_STEPS)
        f32 = s32b.get_state().astype(np.float64)
        s32b.close()
        f64 = finals[("fp64", "mmfd")]
        rel = float(np.linalg.norm(f32 - f64) / np.linalg.norm(f64))
        relm = float(np.linalg.norm(finals[("fp32", "mesofd")] - finals[("fp64", "mesofd")])
                     / np.linalg.norm(finals[("fp64", "mesofd")]))
        meso_vs_mmfd = float(np.abs(finals[("fp64", "mesofd")] - f64).max())
        extra["variants"] = variants
        extra["fp32_rel_l2_vs_fp64_after_10000"] = {"mmfd": rel, "mesofd": relm}
        extra["mesofd_vs_mmfd_fp64_max_abs"] = meso_vs_mmfd

        # HBM-resident point: 8192^2 (2 x 256 MiB > 256 MB Infinity Cache)
        big = I.c2_hill_2d(n=8192)
        sb = c2_solver(M, big, "fp32", "mmfd", stream)
        sb.autotune()
        ms = timed_steps(torch, sb, 1000, reduce_each=False)
        gb = 8192 * 8192 * 1000 / (ms * 1e-3) / 1e9
        extra["hbm_resident_8192_mmfd_fp32"] = dict(glups=round(gb, 2), alg_gbs=round(gb * 8, 1),
                                                    frac_hbm=round(gb * 8 / HBM_PEAK_GBS, 4))
        sb.close()

    cpu = None if args.no_cpu else cpu_baseline(cfg)

    line = {
        "metric": "GLUPS + achieved HBM GB/s (% of peak); batched p50/p99 solve latency",
        "value": round(glups, 2),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D anisotropic linear CDE, D2Q9, MMFD two-level SRT, periodic "
                               "2048x2048, 10000 time steps per step, Gaussian hill + noise",
                   "form": "MMFD", "precision": "fp32", "time_steps_per_step": TIME_STEPS,
                   "nodes": N, "tb_depth": tb},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    s32.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
