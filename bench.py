"""Benchmark of the MesoFD / MMFD time step on one MI355X.

Headline workload (the one the metric is quoted on): the largest single-GPU
configuration, the 2D incompressible NSE, three-level TRT MMFD, D2Q9,
periodic 4096 x 4096 Taylor-Green vortex (Re = 100) with seeded velocity noise,
FP32 state and arithmetic with FP64 reductions, 20 000 time steps per solve.
One benchmark "step" is one full solve: 20 000 time steps, then the FP64
mass / momentum / residual reduction.

Beside it the same JSON line reports
* the FP32 error of the full 20 000-step run against the FP64 run,
* the 2D linear CDE workload (2048^2, 10 000 steps) in every form and
  precision, with its own roofline figures, and an HBM-resident 8192^2 point,
* the theta scheme solved to a residual tolerance,
* the 1D D1Q3 workload (1024 nodes, 1000 steps, dt from the library's
  stability bound),
* the 3D D3Q19 NSE at 512^3 (1000 steps, FP32 error against FP64),
* the source-term workload (Example 1) and the wave equation with Dirichlet
  edges (Example 3 scaled up),
* the batched workload: 256 Burgers grids, one graph launch in FP32, against
  plain per-instance FP64 stepping,
* the serving workload: Poisson arrivals of mixed Burgers / NSE solves under
  a 200 GB and a 2 GB budget, p50 / p99 latency and throughput,
* the oracle on the host cores, all threads and one (CPU baseline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick] [--no-cpu]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# FP32 vector peak, published: 256 CUs x 128 FP32 lanes x 2 flops (fused
# multiply-add) x 2.4 GHz.  (The headline kernel's counters show more than one
# wavefront VALU instruction per CU per clock, so half this figure is no
# ceiling for it.)
VALU_FP32_TFLOPS = 157.3
HEAD_STEPS = 20000  # NSE TGV time steps per solve (headline)
HEAD_SIDE = 4096
NSE_D2Q9_FLOPS_PER_LUP = 230.0  # three-level TRT MMFD, pair form
LCDE_D2Q9_FLOPS_PER_LUP = 30.0  # two-level linear pair form
TIME_STEPS = 10000  # linear CDE workload
N_SIDE = 2048
D0 = 1.0 / 3.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--quick", action="store_true", help="headline only (for profiling)")
    p.add_argument("--no-headline", action="store_true",
                   help="skip the headline (profiling of the other sections; value is then null)")
    p.add_argument("--sections",
                   default="c3err,c2,variants,multiset,theta,theta_mg,nse_theta,general,rect,big,c1,"
                           "nse3d,source,wave,burgers,burgers_theta,batched,serving",
                   help="comma-separated sections to run after the headline")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a 256 MiB device copy (HBM counter calibration)")
    p.add_argument("--serve-requests", type=int, default=2200)
    p.add_argument("--nse3d-steps", type=int, default=1000,
                   help="time steps of the 512^3 NSE section (fewer for profiling runs)")
    p.add_argument("--plan", default="",
                   help="tb,rows,cols: run the headline with this launch plan instead of autotuning "
                        "(used to profile counters on the plan an earlier run chose)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# --------------------------------------------------------------- helpers
def c2_solver(M, cfg, precision, form, stream):
    s = M.Solver("D2Q9", cfg["n"], cfg["dx"], precision, form)
    s.set_equation("lcde", u=cfg["u"], K=cfg["K"], lambda_bar=cfg["lambda_bar"])
    a, _ = M.mfd_preset("srt")
    s.set_scheme("two_level", a, dt=cfg["dt"])
    s.set_stream(stream.cuda_stream)
    s.set_state(cfg["phi0"].astype(s.dtype))
    return s


def timed(torch, fn):
    """GPU time (ms) of fn's work on the current stream, synchronised on both sides."""
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1)


def launch_durations(torch, s, tb, n=1000):
    """Mean GPU duration of one launch of the step kernel, from HIP events
    recorded on the solver's stream around n back-to-back launches that each
    advance `tb` time steps."""
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    s.step(tb * n)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / n


def stored_counters(json_name, kernel_src, tb, w):
    """The committed rocprofv3 counter record of a step kernel
    (profiles/<json_name>), if it was taken on the current kernel source with
    the same steps per launch and window width (the window height changes
    only halo re-reads, which the record states); else None.  Returns a dict
    with hbm_bytes_per_launch, valu_insts_per_launch (or None) and the plan."""
    path = os.path.join(ROOT, "profiles", json_name)
    if not os.path.exists(path):
        return None
    info = json.load(open(path))
    sha = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if info.get("kernel_source_sha256") != sha:
        return None
    for r in [info] + info.get("alternates", []):
        if r.get("time_steps_per_launch") == tb and r.get("window_cols") == w:
            return dict(hbm_bytes_per_launch=r.get("hbm_bytes_per_launch"),
                        valu_insts_per_launch=r.get("valu_insts_per_launch"),
                        plan=[r.get("time_steps_per_launch"), r.get("window_rows"),
                              r.get("window_cols")])
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(c3, budget_s=12.0, one_core_s=8.0):
    """The FP64 oracle (MMFD form) on the host cores, bounded samples of the
    headline workload: all threads, then one thread."""
    from oracle import native as O
    from oracle import scheme as S

    nu, dx, dt = c3["nu"], c3["dx"], c3["dt"]
    s = S.trt_s_for(nu, dx, dt, D0)
    a, ah = S.preset_trt(s)
    spec = dict(lattice="D2Q9", eq="nse", n=c3["n"], dx=dx, dt=dt, rho0=c3["rho0"],
                a=[float(v) for v in a], ah=[float(v) for v in ah], levels=3)
    N = int(np.prod(c3["n"]))

    def run(threads, budget):
        spec["nthreads"] = threads
        cur = c3["state0"].copy()
        prev = cur
        t0 = time.perf_counter()
        steps = 0
        while True:
            cur, prev = O.mmfd_step(spec, cur, prev), cur
            steps += 1
            el = time.perf_counter() - t0
            if el > budget or steps >= 200:
                break
        return N * steps / el / 1e9, steps, el

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    g, st, el = run(threads, budget_s)
    g1, st1, el1 = run(1, one_core_s)
    return dict(value=round(g, 4), unit="GLUPS", cores=threads, kind="oracle",
                cpu_model=cpu_model(), logical_cpus=os.cpu_count(),
                sample="%d three-level TRT NSE MMFD FP64 time steps of the 4096^2 D2Q9 TGV workload "
                       "(%.1f s, %d threads)" % (st, el, threads),
                one_core=dict(value=round(g1, 4), unit="GLUPS", cores=1,
                              sample="%d time steps (%.1f s)" % (st1, el1)))


def two_level_a(M, nu, dx, dt):
    s = 2.0 * nu * dt / (D0 * dx * dx)
    return M.mfd_preset("two_level", s)[0]


def trt_coeffs(M, nu, dx, dt):
    s = 1.0 / (nu / (dt * D0 * (dx / dt) ** 2) + 0.5)
    return M.mfd_preset("trt", s)


# ----------------------------------------------------------- workloads
def bench_variants(M, torch, cfg, stream, N):
    out, finals = {}, {}
    for prec, form, bpl in (("fp64", "mmfd", 16), ("fp32", "mesofd", 72), ("fp64", "mesofd", 144)):
        sv = c2_solver(M, cfg, prec, form, stream)
        sv.autotune()
        ms = timed(torch, lambda: sv.step(TIME_STEPS))
        g = N * TIME_STEPS / (ms * 1e-3) / 1e9
        r = dict(glups=round(g, 2), ms_per_solve=round(ms, 3), plan=list(sv.launch_plan()))
        if form == "mmfd":
            r.update(alg_gbs=round(g * bpl, 1), frac_hbm=round(g * bpl / HBM_PEAK_GBS, 4),
                     bytes_per_lup=bpl)
        else:
            # population form: Q populations in and out per update; a blocked
            # launch carries moments between its steps, so this is a rate
            # the population layout would need, not bytes moved
            r.update(pop_form_bytes_per_lup=bpl, pop_form_equiv_gbs=round(g * bpl, 1))
        out["%s_%s" % (form, prec)] = r
        finals[(prec, form)] = sv.get_state().astype(np.float64)
        sv.close()
    # MesoFD with its populations written at every step (one step per call,
    # so every call stores the b = 9 populations the caller can read back):
    # the cost of streaming the population layout through HBM
    for prec, sz in (("fp32", 4), ("fp64", 8)):
        sv = c2_solver(M, cfg, prec, "mesofd", stream)
        sv.set_blocking(1)
        nstep = 300

        def run():
            for _ in range(nstep):
                sv.step(1)
        run()
        ms = timed(torch, run)
        g = N * nstep / (ms * 1e-3) / 1e9
        out["mesofd_populations_every_step_" + prec] = dict(
            glups=round(g, 2), steps=nstep, populations_written_gbs=round(g * 9 * sz, 1),
            pop_form_bytes_per_lup=2 * 9 * sz, frac_hbm_pop_form=round(g * 18 * sz / HBM_PEAK_GBS, 4))
        sv.close()
    s32 = c2_solver(M, cfg, "fp32", "mmfd", stream)
    s32.step(TIME_STEPS)
    f32 = s32.get_state().astype(np.float64)
    s32.close()
    f64 = finals[("fp64", "mmfd")]
    err = dict(mmfd=float(np.linalg.norm(f32 - f64) / np.linalg.norm(f64)),
               mesofd=float(np.linalg.norm(finals[("fp32", "mesofd")] - finals[("fp64", "mesofd")])
                            / np.linalg.norm(finals[("fp64", "mesofd")])))
    meso_vs_mmfd = float(np.abs(finals[("fp64", "mesofd")] - f64).max())
    # the three-level scheme of Example 1 Case 3 (a = 7/8, 0, 1/8; ah = 1/8,
    # 0, -1/8) on the same workload, both levels starting from phi0
    f3 = {}
    for prec in ("fp32", "fp64"):
        sv = M.Solver("D2Q9", cfg["n"], cfg["dx"], prec, "mmfd")
        sv.set_equation("lcde", u=cfg["u"], K=cfg["K"], lambda_bar=cfg["lambda_bar"])
        sv.set_scheme("three_level", (7 / 8, 0.0, 1 / 8), (1 / 8, 0.0, -1 / 8), dt=cfg["dt"])
        sv.set_stream(stream.cuda_stream)
        sv.set_state(cfg["phi0"].astype(sv.dtype))
        sv.autotune()
        ms = timed(torch, lambda: sv.step(TIME_STEPS))
        g = N * TIME_STEPS / (ms * 1e-3) / 1e9
        bpl = 3 * (8 if prec == "fp64" else 4)  # read t and t - dt, write t + dt
        out["mmfd_three_level_" + prec] = dict(glups=round(g, 2), ms_per_solve=round(ms, 3),
                                               plan=list(sv.launch_plan()), alg_gbs=round(g * bpl, 1),
                                               frac_hbm=round(g * bpl / HBM_PEAK_GBS, 4),
                                               bytes_per_lup=bpl)
        f3[prec] = sv.get_state().astype(np.float64)
        sv.close()
    err["mmfd_three_level"] = float(np.linalg.norm(f3["fp32"] - f3["fp64"]) / np.linalg.norm(f3["fp64"]))
    return out, err, meso_vs_mmfd


def bench_theta(M, torch, cfg, stream, N, theta=0.5, steps=1000, chunk=8, cap=64):
    """theta scheme (linear CDE, SRT coefficients) on the 2048^2 workload,
    each step solved to a residual tolerance (binary64 1e-12, binary32 1e-6;
    Jacobi sweeps checked every `chunk`, at most `cap`): GLUPS at convergence,
    sweeps per step, the FP32 error against the FP64 run of the same steps."""
    out = {}
    finals = {}
    for prec, tol in (("fp32", 1e-6), ("fp64", 1e-12)):
        s = M.Solver("D2Q9", cfg["n"], cfg["dx"], prec, "mmfd")
        s.set_equation("lcde", u=cfg["u"], K=cfg["K"], lambda_bar=cfg["lambda_bar"])
        s.set_scheme("theta", M.mfd_preset("srt")[0], theta=theta, theta_iters=cap, dt=cfg["dt"])
        s.set_theta_tolerance(tol, chunk)
        s.set_stream(stream.cuda_stream)
        s.set_state(cfg["phi0"].astype(s.dtype))
        s.step(10)
        s.set_state(cfg["phi0"].astype(s.dtype))
        s.theta_stats(reset=True)
        ms = timed(torch, lambda: s.step(steps))
        st = s.theta_stats()
        finals[prec] = s.get_state().astype(np.float64)
        s.close()
        g = N * steps / (ms * 1e-3) / 1e9
        sw = st["total_sweeps"] / max(st["steps"], 1)
        out[prec] = dict(glups=round(g, 2), tolerance=tol, sweeps_per_step=round(sw, 2),
                         max_sweeps=st["max_sweeps"], steps_stopped_by_cap=st["unconverged"],
                         sweep_glups=round(g * sw, 2))
    out.update(theta=theta, chunk_sweeps=chunk, sweep_cap=cap, steps=steps,
               fp32_rel_l2_vs_fp64=float(np.linalg.norm(finals["fp32"] - finals["fp64"])
                                         / np.linalg.norm(finals["fp64"])))
    return out


def bench_theta_mg(M, torch, cfg, stream, N, theta=0.5, dt_factor=32.0, steps=20):
    """theta scheme of the 2048^2 linear CDE at dt_factor times the explicit
    time step, where Jacobi sweeps need hundreds per step: the same steps
    solved to the same residual tolerance by Jacobi sweeps (device-decided
    chunks) and by multigrid V(2,2) cycles over every level the grid allows.
    GLUPS count time steps; FP32 error against the FP64 multigrid run, and
    the FP64 multigrid result against the FP64 Jacobi one."""
    out, finals = {}, {}
    dt = cfg["dt"] * dt_factor
    for solver, prec, tol, cap, chunk in (("jacobi", "fp64", 1e-10, 4096, 16),
                                          ("multigrid", "fp64", 1e-10, 40, 0),
                                          ("jacobi", "fp32", 1e-5, 4096, 16),
                                          ("multigrid", "fp32", 1e-5, 40, 0)):
        s = M.Solver("D2Q9", cfg["n"], cfg["dx"], prec, "mmfd")
        s.set_equation("lcde", u=cfg["u"], K=cfg["K"], lambda_bar=cfg["lambda_bar"])
        s.set_scheme("theta", M.mfd_preset("srt")[0], theta=theta, theta_iters=cap, dt=dt)
        s.set_theta_tolerance(tol, chunk)
        if solver == "multigrid":
            s.set_theta_multigrid(-1, 2, 2)
        s.set_stream(stream.cuda_stream)
        s.set_state(cfg["phi0"].astype(s.dtype))
        s.step(2)
        s.set_state(cfg["phi0"].astype(s.dtype))
        s.theta_stats(reset=True)
        ms = timed(torch, lambda: s.step(steps))
        st = s.theta_stats()
        finals[solver, prec] = s.get_state().astype(np.float64)
        s.close()
        g = N * steps / (ms * 1e-3) / 1e9
        it = st["total_sweeps"] / max(st["steps"], 1)
        out["%s_%s" % (solver, prec)] = dict(
            glups=round(g, 3), ms_per_step=round(ms / steps, 3), tolerance=tol,
            **{("cycles_per_step" if solver == "multigrid" else "sweeps_per_step"): round(it, 2)},
            steps_stopped_by_cap=st["unconverged"])
    ref = finals["multigrid", "fp64"]
    out.update(theta=theta, dt_over_explicit=dt_factor, steps=steps,
               multigrid_vs_jacobi_fp64_rel_l2=float(np.linalg.norm(ref - finals["jacobi", "fp64"])
                                                     / np.linalg.norm(ref)),
               fp32_multigrid_rel_l2_vs_fp64=float(np.linalg.norm(finals["multigrid", "fp32"] - ref)
                                                   / np.linalg.norm(ref)),
               speedup_fp64=round(out["multigrid_fp64"]["glups"] / out["jacobi_fp64"]["glups"], 2),
               speedup_fp32=round(out["multigrid_fp32"]["glups"] / out["jacobi_fp32"]["glups"], 2))
    return out


def bench_big(M, torch, I, stream):
    big = I.c2_hill_2d(n=8192)
    sb = c2_solver(M, big, "fp32", "mmfd", stream)
    sb.autotune()
    ms = timed(torch, lambda: sb.step(1000))
    g = 8192 * 8192 * 1000 / (ms * 1e-3) / 1e9
    sb.close()
    return dict(glups=round(g, 2), alg_gbs=round(g * 8, 1), frac_hbm=round(g * 8 / HBM_PEAK_GBS, 4))


def bench_c1(M, torch, I, stream):
    c1 = I.c1_linear_1d()
    # dt = half the library's Eq. (LMMFD-2-3) bound (the recipe's 25 * 2^-20)
    bound, exact = M.mfd_max_stable_dt("D1Q3", c1["dx"], c1["u"], c1["D"], n=c1["n"])
    c1["dt"] = 0.5 * bound
    res = dict(dt=c1["dt"], dt_bound_sufficient=bound, dt_bound_exact_modes=exact)
    for form in ("mmfd", "mesofd"):
        s = M.Solver("D1Q3", c1["n"], c1["dx"], "fp64", form)
        s.set_equation("lcde", u=c1["u"], K=c1["K"])
        sp = 2 * c1["D"] * c1["dt"] / (D0 * c1["dx"] ** 2)
        s.set_scheme("two_level", M.mfd_preset("two_level", sp)[0], dt=c1["dt"])
        s.set_stream(stream.cuda_stream)
        s.set_state(c1["phi0"])
        s.step(c1["steps"])  # warm-up
        s.set_state(c1["phi0"])
        ms = timed(torch, lambda: s.step(c1["steps"]))
        res[form + "_fp64_us_per_1000_steps"] = round(ms * 1e3, 1)
        s.close()
    return res


def bench_source(M, torch, I, stream, steps=500):
    """Example 1 (linear CDE with the source R, three-level Case 2 with the
    source coefficients b_-1 = 3/2, bh_-1 = -1/2) on a 2048^2 grid, FP64 and
    FP32: GLUPS of step + source launches, the FP32 error against FP64 and
    the FP64 run's GRE against the exact solution."""
    ex = I.example1_source_2d(n=N_SIDE)
    a, ah = (7 / 8, 1 / 4, -1 / 8), (1 / 8, -1 / 4, 1 / 8)
    out, finals = {}, {}
    for prec, form in (("fp64", "mmfd"), ("fp32", "mmfd"), ("fp64", "mesofd"), ("fp32", "mesofd")):
        s = M.Solver("D2Q9", ex["n"], ex["dx"], prec, form)
        s.set_equation("lcde", u=ex["u"], K=ex["K"], lambda_bar=1)
        s.set_scheme("three_level", a, ah, dt=ex["dt"])
        s.set_stream(stream.cuda_stream)

        def start():
            s.set_state(ex["phi0"].astype(s.dtype))
            s.set_state(ex["phim"].astype(s.dtype), level=1)
            s.set_source(ex["G"], ex["lam"], (1.5, 0.0, 0.0), (-0.5, 0.0, 0.0), ex["u"])
        start()
        if form == "mmfd":
            s.autotune()  # blocked source plans (G staged once per launch) or single steps
            start()
        s.step(20)
        start()
        ms = timed(torch, lambda: s.step(steps))
        plan = s.launch_plan()
        finals[prec, form] = s.get_state().astype(np.float64)
        s.close()
        g = ex["n"][0] * ex["n"][1] * steps / (ms * 1e-3) / 1e9
        es = 8 if prec == "fp64" else 4
        key = prec if form == "mmfd" else "mesofd_" + prec
        if form == "mmfd":
            bpl = 4 * es  # read t, t - dt and G; write t + dt
            out[key] = dict(glups=round(g, 2), alg_gbs=round(g * bpl, 1),
                            frac_hbm_algorithmic=round(g * bpl / HBM_PEAK_GBS, 4),
                            bytes_per_lup=bpl, time_steps_per_launch=plan[0],
                            window_rows=plan[1], window_cols=plan[2])
        else:
            # the population form's own bytes: read and write the 9 populations, read G
            bpl = (2 * 9 + 1) * es
            out[key] = dict(glups=round(g, 2), pop_form_bytes_per_lup=bpl,
                            pop_form_equiv_gbs=round(g * bpl, 1))
    exact = ex["exact"](steps * ex["dt"])
    f64 = finals["fp64", "mmfd"]
    out.update(steps=steps, scheme="three-level (7/8, 1/4, -1/8 | 1/8, -1/4, 1/8), b_-1 = 3/2, bh_-1 = -1/2",
               fp32_rel_l2_vs_fp64=float(np.linalg.norm(finals["fp32", "mmfd"] - f64) / np.linalg.norm(f64)),
               mesofd_vs_mmfd_fp64_max_abs=float(np.abs(finals["fp64", "mesofd"] - f64).max()),
               fp64_gre_vs_exact=float(np.abs(f64 - exact).sum() / np.abs(exact).sum()))
    return out


def _nse_solver(M, lat, c, precision, stream):
    a, ah = trt_coeffs(M, c["nu"], c["dx"], c["dt"])
    s = M.Solver(lat, c["n"], c["dx"], precision, "mmfd")
    s.set_equation("nse", rho0=c["rho0"])
    s.set_scheme("three_level", a, ah, dt=c["dt"])
    s.set_stream(stream.cuda_stream)
    return s


def _rel_l2_dev(torch, a, b):
    """Relative L2 distance of two device tensors, in binary64."""
    a = a.double()
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def bench_nse3d(M, torch, I, stream, steps=1000):
    """Three-level TRT NSE on D3Q19 at 512^3, 1000 time steps in FP32 (after
    the autotuner), and the FP32 error against the FP64 run of the same steps
    from the same (binary32-rounded) start."""
    c = I.tgv_3d(n=512, dtype=np.float32)
    x0 = torch.from_numpy(np.ascontiguousarray(c["state0"], dtype=np.float32)).to("cuda")
    del c["state0"]
    nodes = int(np.prod(c["n"]))
    s = _nse_solver(M, "D3Q19", c, "fp32", stream)
    s.set_state(x0)
    s.autotune()
    plan = s.launch_plan()
    s.step(2)
    s.set_state(x0)
    ms = timed(torch, lambda: s.step(steps))
    g = nodes * steps / (ms * 1e-3) / 1e9
    y32 = torch.empty_like(x0)
    s.get_state(out=y32)
    s.close()
    s64 = _nse_solver(M, "D3Q19", c, "fp64", stream)
    x64 = x0.double()
    del x0
    s64.set_state(x64)
    ms64 = timed(torch, lambda: s64.step(steps))
    y64 = torch.empty_like(x64)
    s64.get_state(out=y64)
    s64.close()
    torch.cuda.synchronize()
    bpl = 48
    res = dict(glups=round(g, 2), fp64_glups=round(nodes * steps / (ms64 * 1e-3) / 1e9, 2),
               alg_gbs=round(g * bpl, 1), frac_hbm_algorithmic=round(g * bpl / HBM_PEAK_GBS, 4),
               bytes_per_lup=bpl, steps=steps, plan=list(plan),
               fp32_rel_l2_vs_fp64=_rel_l2_dev(torch, y32, y64))
    del x64, y32, y64
    torch.cuda.empty_cache()
    return res


def bench_c3_error(M, torch, c3, x0, stream, steps=HEAD_STEPS):
    """FP32 error of the headline workload after its full run: the FP32 solve
    of `steps` time steps against the FP64 solve from the same
    (binary32-rounded) start, relative L2 over all fields."""
    out = {}
    ys = {}
    for prec in ("fp32", "fp64"):
        s = _nse_solver(M, "D2Q9", c3, prec, stream)
        x = x0 if prec == "fp32" else x0.double()
        s.set_state(x)
        ms = timed(torch, lambda: s.step(steps))
        y = torch.empty_like(x)
        s.get_state(out=y)
        sums = s.reduce()
        s.close()
        ys[prec] = y
        out[prec + "_glups"] = round(int(np.prod(c3["n"])) * steps / (ms * 1e-3) / 1e9, 2)
        out[prec + "_mass_momentum"] = [float(v) for v in sums[0][:3]]
    out["fp32_rel_l2_vs_fp64"] = _rel_l2_dev(torch, ys["fp32"], ys["fp64"])
    out["steps"] = steps
    del ys
    torch.cuda.empty_cache()
    return out


def bench_wave(M, torch, stream, nx=4095):
    """The wave equation of Example 3 scaled up: phi = exp(x + y + t) on
    [0,1]^2 with (nx + 1)^2 nodes, dt = dx / 2 (N_t = 2 N_x), Dirichlet edges
    from the exact solution, the special first step, D2Q9, beta = 3/4,
    gamma = 1/2 (Case 3), T = 1.  FP32 and FP64: GLUPS of the three-level
    steps (64-column blocked windows), the GRE against the exact solution and
    the FP32 error against FP64."""
    import math
    n = (nx + 1, nx + 1)
    dx = 1.0 / nx
    dt = dx / 2.0
    steps = 2 * nx
    x = np.arange(nx + 1) * dx
    G = np.exp(x[None, :] + x[:, None]).ravel()
    gamma, beta = 0.5, 0.75
    a, ah = (gamma, 2 * (1 - gamma), gamma), (0.0, -1.0, 0.0)
    out, fin = {}, {}
    N = n[0] * n[1]
    for prec in ("fp32", "fp64"):
        s = M.Solver("D2Q9", n, dx, prec, "mmfd", boundary="dirichlet")
        s.set_equation("wave", beta=beta)
        s.set_scheme("three_level", a, ah, dt=dt)
        s.set_stream(stream.cuda_stream)
        s.set_boundary(G, 1.0)

        def start():
            s.set_state(G.astype(s.dtype))
            s.wave_start(G)
        start()
        s.autotune()
        start()
        ms = timed(torch, lambda: s.step(steps - 1))
        plan = s.launch_plan()
        fin[prec] = s.get_state().astype(np.float64)
        s.close()
        g = N * (steps - 1) / (ms * 1e-3) / 1e9
        bpl = 3 * (4 if prec == "fp32" else 8)
        ex = (G * math.e).reshape(n)[1:-1, 1:-1]
        gre = float(np.abs(fin[prec].reshape(n)[1:-1, 1:-1] - ex).sum() / np.abs(ex).sum())
        out[prec] = dict(glups=round(g, 2), alg_gbs=round(g * bpl, 1),
                         frac_hbm_algorithmic=round(g * bpl / HBM_PEAK_GBS, 4), bytes_per_lup=bpl,
                         plan=list(plan), gre_vs_exact=gre)
    out.update(nodes=N, steps=steps, scheme="a = (1/2, 1, 1/2), ah = (0, -1, 0), beta = 3/4",
               fp32_rel_l2_vs_fp64=float(np.linalg.norm(fin["fp32"] - fin["fp64"])
                                         / np.linalg.norm(fin["fp64"])))
    return out


def bench_burgers_single(M, torch, I, stream):
    """One 2048^2 Burgers grid (the batched workload's recipe at its largest
    side class), FP32 MMFD, 1000 steps."""
    rng = np.random.default_rng(6)
    c = I.burgers_instance(rng, side_lo=2048, side_hi=2048, steps_lo=1000, steps_hi=1000)
    s = M.Solver("D2Q9", c["n"], c["dx"], "fp32", "mmfd")
    s.set_equation("burgers")
    s.set_scheme("two_level", two_level_a(M, c["nu"], c["dx"], c["dt"]), dt=c["dt"])
    s.set_stream(stream.cuda_stream)
    s.set_state(c["phi0"].astype(np.float32))
    s.autotune()
    tb, h, w = s.launch_plan()
    s.step(50)
    ms = timed(torch, lambda: s.step(1000))
    s.close()
    g = 2048 * 2048 * 1000 / (ms * 1e-3) / 1e9
    return dict(glups=round(g, 2), alg_gbs=round(g * 8, 1), frac_hbm=round(g * 8 / HBM_PEAK_GBS, 4),
                bytes_per_lup=8, time_steps_per_launch=tb, window_rows=h, window_cols=w)


def bench_burgers_theta(M, torch, I, stream, theta=0.5, steps=200, chunk=4, cap=64):
    """theta scheme for Burgers' equation (Picard iteration with the Jacobi
    splitting of the linear even part) on one 2048^2 grid of the batched
    workload's recipe, dt four times its explicit step, each step solved to a
    tolerance (binary64 1e-12, binary32 2e-7: a stopping error of 1e-6 per
    step accumulates to ~1e-4 over the run): GLUPS at convergence, sweeps per
    step, FP32 error against the FP64 run of the same steps."""
    rng = np.random.default_rng(6)
    c = I.burgers_instance(rng, side_lo=2048, side_hi=2048, steps_lo=steps, steps_hi=steps)
    dt = 4.0 * c["dt"]
    sp = 2 * c["nu"] * dt / ((1.0 / 3.0) * c["dx"] ** 2)
    a = M.mfd_preset("two_level", sp)[0]
    out, finals = {}, {}
    N = 2048 * 2048
    for prec, tol in (("fp32", 2e-7), ("fp64", 1e-12)):
        s = M.Solver("D2Q9", c["n"], c["dx"], prec, "mmfd")
        s.set_equation("burgers")
        s.set_scheme("theta", a, theta=theta, theta_iters=cap, dt=dt)
        s.set_theta_tolerance(tol, chunk)
        s.set_stream(stream.cuda_stream)
        s.set_state(c["phi0"].astype(s.dtype))
        s.step(5)
        s.set_state(c["phi0"].astype(s.dtype))
        s.theta_stats(reset=True)
        ms = timed(torch, lambda: s.step(steps))
        st = s.theta_stats()
        finals[prec] = s.get_state().astype(np.float64)
        s.close()
        g = N * steps / (ms * 1e-3) / 1e9
        sw = st["total_sweeps"] / max(st["steps"], 1)
        out[prec] = dict(glups=round(g, 2), tolerance=tol, sweeps_per_step=round(sw, 2),
                         max_sweeps=st["max_sweeps"], steps_stopped_by_cap=st["unconverged"],
                         sweep_glups=round(g * sw, 2))
    out.update(theta=theta, dt_over_explicit=4.0, chunk_sweeps=chunk, sweep_cap=cap, steps=steps,
               fp32_rel_l2_vs_fp64=float(np.linalg.norm(finals["fp32"] - finals["fp64"])
                                         / np.linalg.norm(finals["fp64"])))
    return out


def bench_nse_theta(M, torch, I, stream, theta=0.5, steps=100, chunk=4, cap=64, courant=0.2):
    """theta scheme for the 2D NSE (Picard sweeps with the linear parts'
    own-node coefficient split per field) on the 1024^2 Taylor-Green vortex
    with dt = 0.2 dx / U0 (four times the explicit recipe's), density set
    s = 1 and momentum set s = 1 / (nu dt / (d0 dx^2) + 1/2), each step solved
    to a tolerance (binary64 1e-12, binary32 1e-6): GLUPS at convergence,
    sweeps per step, FP32 error against the FP64 run of the same steps."""
    c = I.tgv_2d(n=1024, courant=courant)
    s_j = 1.0 / (c["nu"] * c["dt"] / (D0 * c["dx"] ** 2) + 0.5)
    fam = lambda s: ((s + 1) / 2, 1 - s, (s - 1) / 2)
    N = 1024 * 1024
    out, finals = {}, {}
    for prec, tol in (("fp32", 1e-6), ("fp64", 1e-12)):
        sv = M.Solver("D2Q9", c["n"], c["dx"], prec, "mmfd")
        sv.set_equation("nse", rho0=c["rho0"])
        sv.set_scheme("theta", fam(1.0), ab=fam(s_j), theta=theta, theta_iters=cap, dt=c["dt"])
        sv.set_theta_tolerance(tol, chunk)
        sv.set_stream(stream.cuda_stream)
        sv.set_state(c["state0"].astype(sv.dtype))
        sv.step(3)
        sv.set_state(c["state0"].astype(sv.dtype))
        sv.theta_stats(reset=True)
        ms = timed(torch, lambda: sv.step(steps))
        st = sv.theta_stats()
        finals[prec] = sv.get_state().astype(np.float64)
        sv.close()
        g = N * steps / (ms * 1e-3) / 1e9
        sw = st["total_sweeps"] / max(st["steps"], 1)
        out[prec] = dict(glups=round(g, 3), tolerance=tol, sweeps_per_step=round(sw, 2),
                         max_sweeps=st["max_sweeps"], steps_stopped_by_cap=st["unconverged"],
                         sweep_glups=round(g * sw, 2))
    out.update(theta=theta, courant=courant, momentum_s=round(s_j, 4), chunk_sweeps=chunk,
               sweep_cap=cap, steps=steps,
               fp32_rel_l2_vs_fp64=float(np.linalg.norm(finals["fp32"] - finals["fp64"])
                                         / np.linalg.norm(finals["fp64"])))
    return out


def bench_general(M, torch, I, stream):
    """The general-scheme solver (mfd_general_*): the rD3Q27 linear CDE at
    256^3 (reach 1, one level), the 2048^2 rD2Q9 linear CDE with reach 2 and
    two levels, and the 1024^2 rD2Q9 Taylor-Green NSE with reach 2; GLUPS of
    FP32 and FP64 and the FP32 error against FP64 after the same steps.
    Tables: A00 = 1 and A10 = A11 = -1 (Eq. (4-2-00a)); each row k = -m..m."""
    one = np.array([[1.0, 0.0, 0.0]])                                  # A22 = 1/2
    two = np.array([[0.2, 0.6, 0.2, 0.0, 0.0], [-0.05, 0.1, -0.05, 0.0, 0.0]])  # A22 = 0.65
    wide = np.array([[0.25, 0.5, 0.25, 0.0, 0.0]])                     # A22 = 3/4
    tgv = I.tgv_2d(n=1024)
    cases = [
        ("lcde_d3q27_256_m1", "D3Q27", (256, 256, 256), one, 20),
        ("lcde_d2q9_2048_m2_n2", "D2Q9", (2048, 2048), two, 100),
        ("nse_d2q9_1024_m2", "D2Q9", (1024, 1024), wide, 100),
    ]
    out = {}
    for name, lat, n, a, steps in cases:
        N = int(np.prod(n))
        dim = len(n)
        nse = name.startswith("nse")
        if nse:
            state = tgv["state0"]
        else:
            x = np.indices(tuple(reversed(n)), dtype=np.float64)
            state = np.exp(sum(np.cos(2 * np.pi * x[i] / n[dim - 1 - i]) for i in range(dim))).ravel()
            del x
        res, fin = {}, {}
        for prec in ("fp32", "fp64"):
            if nse:
                g = M.General(lat, n, tgv["dx"], a, tgv["dt"], precision=prec, eq="nse", ab=a,
                              rho0=tgv["rho0"])
            else:
                g = M.General(lat, n, 1.0, a, 1.0, u=[0.05, -0.03, 0.02][:dim],
                              K=(np.eye(dim) * 0.1).tolist(), lambda_bar=1, precision=prec)
            g.set_stream(stream.cuda_stream)
            for l in range(a.shape[0]):
                g.set_level(l, state)
            g.step(2)
            for l in range(a.shape[0]):
                g.set_level(l, state)
            ms = timed(torch, lambda: g.step(steps))
            fin[prec] = g.get_level(0).astype(np.float64)
            g.close()
            res[prec + "_glups"] = round(N * steps / (ms * 1e-3) / 1e9, 2)
        res.update(steps=steps, reach=(a.shape[1] - 1) // 2, levels=a.shape[0],
                   fp32_rel_l2_vs_fp64=float(np.linalg.norm(fin["fp32"] - fin["fp64"])
                                             / np.linalg.norm(fin["fp64"])))
        out[name] = res
    return out


def bench_rect(M, torch, cfg, stream, N, steps=1000):
    """The 2048^2 linear CDE on a rectangular rD2Q9 lattice (dy = 2 dx,
    d0 = (1/3, 1/4)), autotuned plan: GLUPS of FP32 and FP64 and the FP32
    error against FP64 (the kernels are the square lattice's)."""
    out, fin = {}, {}
    for prec in ("fp32", "fp64"):
        s = M.Solver("D2Q9", cfg["n"], cfg["dx"], prec, "mmfd")
        s.set_rectangular((cfg["dx"], 2 * cfg["dx"]), (1.0 / 3.0, 0.25))
        s.set_equation("lcde", u=cfg["u"], K=cfg["K"], lambda_bar=cfg["lambda_bar"])
        s.set_scheme("two_level", M.mfd_preset("srt")[0], dt=cfg["dt"])
        s.set_stream(stream.cuda_stream)
        s.set_state(cfg["phi0"].astype(s.dtype))
        s.autotune()
        s.set_state(cfg["phi0"].astype(s.dtype))
        ms = timed(torch, lambda: s.step(steps))
        fin[prec] = s.get_state().astype(np.float64)
        plan = s.launch_plan()
        s.close()
        out[prec] = dict(glups=round(N * steps / (ms * 1e-3) / 1e9, 2), plan=list(plan))
    out.update(steps=steps, spacing=[cfg["dx"], 2 * cfg["dx"]], d0=[1.0 / 3.0, 0.25],
               fp32_rel_l2_vs_fp64=float(np.linalg.norm(fin["fp32"] - fin["fp64"])
                                         / np.linalg.norm(fin["fp64"])))
    return out


def bench_multiset(M, torch, cfg, stream, N, steps=1000):
    """Multiple-set (TRT-type) two-level linear CDE, Eq. (2-2-1b), on the
    2048^2 workload: base set SRT (a_-1 = 1), even set (1/2, 0, 1/2) and odd
    set (3/4, 0, -1/4), which keep SRT's a_1 + a_-1 and a_1 - a_-1 (the
    transport coefficients unchanged, so the run is stable at the same dt).
    GLUPS (autotuned plan), FP32 error against FP64 after the run."""
    a = M.mfd_preset("srt")[0]
    ae = (0.5, 0.0, 0.5)
    ao = (0.75, 0.0, -0.25)
    out, finals = {}, {}
    for prec in ("fp32", "fp64"):
        s = M.Solver("D2Q9", cfg["n"], cfg["dx"], prec, "mmfd")
        s.set_equation("lcde", u=cfg["u"], K=cfg["K"], lambda_bar=cfg["lambda_bar"])
        s.set_scheme_sets("two_level", a, ae, ao, dt=cfg["dt"])
        s.set_stream(stream.cuda_stream)
        s.set_state(cfg["phi0"].astype(s.dtype))
        s.autotune()
        s.set_state(cfg["phi0"].astype(s.dtype))
        ms = timed(torch, lambda: s.step(steps))
        plan = s.launch_plan()
        finals[prec] = s.get_state().astype(np.float64)
        s.close()
        g = N * steps / (ms * 1e-3) / 1e9
        bpl = 2 * (4 if prec == "fp32" else 8)
        out[prec] = dict(glups=round(g, 2), alg_gbs=round(g * bpl, 1),
                         frac_hbm_algorithmic=round(g * bpl / HBM_PEAK_GBS, 4),
                         time_steps_per_launch=plan[0], window_rows=plan[1], window_cols=plan[2])
    out.update(steps=steps, base=a, even=ae, odd=ao,
               fp32_rel_l2_vs_fp64=float(np.linalg.norm(finals["fp32"] - finals["fp64"])
                                         / np.linalg.norm(finals["fp64"])))
    return out


def bench_batched(M, torch, I, stream):
    insts = I.c4_batch(256, seed=4)
    lups = sum(int(np.prod(c["n"])) * c["steps"] for c in insts)

    def make(c, prec):
        s = M.Solver("D2Q9", c["n"], c["dx"], prec, "mmfd")
        s.set_equation("burgers")
        s.set_scheme("two_level", two_level_a(M, c["nu"], c["dx"], c["dt"]), dt=c["dt"])
        s.set_stream(stream.cuda_stream)
        s.set_state(c["phi0"].astype(s.dtype))
        return s

    s32 = [make(c, "fp32") for c in insts]
    b = M.Batch(stream.cuda_stream, use_graph=True)
    for s, c in zip(s32, insts):
        b.add(s, c["steps"])
    t0 = time.perf_counter()
    b.autotune()  # launch plan of the group (steps per launch, window rows)
    tune_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    b.run()
    b.wait()
    first_s = time.perf_counter() - t0  # includes graph capture + instantiation
    for s, c in zip(s32, insts):
        s.set_state(c["phi0"].astype(np.float32))
    ms32 = timed(torch, lambda: b.run())
    st = b.stats()
    plan = b.plan(0)
    # plain per-instance FP64 stepping: one launch per step per instance
    s64 = [make(c, "fp64") for c in insts]
    for s in s64:
        s.set_blocking(1)
    ms64 = timed(torch, lambda: [s.step(c["steps"]) for s, c in zip(s64, insts)])
    errs, errs0, decay = [], [], []
    for a32, a64, c in zip(s32, s64, insts):
        x = a32.get_state().astype(np.float64)
        y = a64.get_state()
        n0 = np.linalg.norm(c["phi0"])
        errs.append(float(np.linalg.norm(x - y) / np.linalg.norm(y)))
        errs0.append(float(np.linalg.norm(x - y) / n0))
        decay.append(float(np.linalg.norm(y) / n0))
    worst = int(np.argmax(errs))
    for s in s32 + s64:
        s.close()
    b.close()
    g32 = lups / (ms32 * 1e-3) / 1e9
    g64 = lups / (ms64 * 1e-3) / 1e9
    return dict(instances=len(insts), lups=lups, graph_launches=st["launches"], tiles=st["tiles"],
                plan=dict(time_steps_per_launch=plan[0], window_rows=plan[1], window_cols=plan[2]),
                autotune_s=round(tune_s, 3),
                fp32_graph_ms=round(ms32, 2), fp32_glups=round(g32, 2),
                fp32_first_run_incl_capture_s=round(first_s, 3),
                fp64_per_instance_ms=round(ms64, 2), fp64_glups=round(g64, 2),
                speedup_vs_fp64_per_instance=round(ms64 / ms32, 2),
                fp32_rel_l2_vs_fp64_max=max(errs), fp32_rel_l2_vs_fp64_median=float(np.median(errs)),
                fp32_err_over_initial_norm_max=max(errs0),
                worst_instance=dict(side=insts[worst]["n"][0], steps=insts[worst]["steps"],
                                    final_over_initial_norm=decay[worst]))


def bench_tiny_batch(M, torch, I, stream, count=512):
    """Many small grids: 512 Burgers grids of the batched recipe with sides
    log-uniform in [16, 64] and 200 .. 2000 steps, FP32, one graph per run:
    the LDS-resident path (every grid within 4096 nodes: all steps in one
    workgroup) against the windowed launches (resident path off, autotuned
    plan).  Both give the solo results bit for bit."""
    insts = I.c4_batch(count, seed=7, side_lo=16, side_hi=64, steps_lo=200, steps_hi=2000)
    lups = sum(int(np.prod(c["n"])) * c["steps"] for c in insts)
    out = {}
    finals = {}
    for name, res in (("resident", 4096), ("windowed", 0)):
        ss = []
        b = M.Batch(stream.cuda_stream, use_graph=True)
        b.set_resident(res)
        for c in insts:
            s = M.Solver("D2Q9", c["n"], c["dx"], "fp32", "mmfd")
            s.set_equation("burgers")
            s.set_scheme("two_level", two_level_a(M, c["nu"], c["dx"], c["dt"]), dt=c["dt"])
            s.set_stream(stream.cuda_stream)
            s.set_state(c["phi0"].astype(np.float32))
            b.add(s, c["steps"])
            ss.append(s)
        if not res:
            b.autotune()
        b.run()
        b.wait()  # capture and first run
        for s, c in zip(ss, insts):
            s.set_state(c["phi0"].astype(np.float32))
        ms = timed(torch, lambda: b.run())
        st = b.stats()
        finals[name] = [s.get_state() for s in ss]
        out[name] = dict(glups=round(lups / (ms * 1e-3) / 1e9, 2), ms=round(ms, 2),
                         launches=st["launches"], resident_instances=b.resident())
        b.close()
        for s in ss:
            s.close()
    out["identical"] = all(np.array_equal(a, b) for a, b in zip(finals["resident"], finals["windowed"]))
    out.update(instances=count, lups=lups)
    return out


def serving_requests(M, I, n_total, rate=200.0, warm=200):
    """The serving trace's requests with their initial states (built once,
    shared by the runs under different budgets)."""
    from concurrent.futures import ThreadPoolExecutor

    trace = I.serving_trace(count=n_total - warm, warmup=warm, rate=rate)
    reqs = []
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        states = list(ex.map(I.serving_request_state, trace))
    for r, inst in zip(trace, states):
        dx, dt = inst["dx"], inst["dt"]
        if r["kind"] == "burgers":
            st = inst["phi0"].astype(np.float32)
            a, ah, kind, eq, rho0 = two_level_a(M, inst["nu"], dx, dt), None, "two_level", "burgers", 0.0
        else:
            st = inst["state0"].astype(np.float32)
            a, ah = trt_coeffs(M, inst["nu"], dx, dt)
            kind, eq, rho0 = "three_level", "nse", inst["rho0"]
        reqs.append(dict(r=r, st=st, a=a, ah=ah, kind=kind, eq=eq, rho0=rho0, n=inst["n"], dx=dx,
                         dt=dt))
    return reqs, time.perf_counter() - t0, trace


def bench_serving(M, reqs_all, gen_s, n_warm, rate=200.0, quantum=50, budget=200 * 10 ** 9):
    reqs = []
    for q in reqs_all:
        out = np.empty_like(q["st"])
        req = M.make_request("D2Q9", q["eq"], q["n"], q["dx"], q["dt"], q["a"], q["r"]["steps"], q["st"],
                             ah=q["ah"], kind=q["kind"], precision="fp32", rho0=q["rho0"],
                             result_out=out, exclude=q["r"]["warmup"])
        reqs.append((q["r"], req, q["st"], out))
    srv = M.Server(hbm_budget_bytes=budget, max_slots=1024, quantum_steps=quantum)
    M.memory_stats(reset_peak=True)
    base, _ = M.memory_stats()
    tickets = []

    def submitter():
        start = time.perf_counter()
        for r, req, st, out in reqs:
            delay = start + r["arrival"] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(req, keep=(st, out)))

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    srv.drain(600)
    _, peak = M.memory_stats()
    stats = srv.stats()
    fails = sum(1 for t in tickets if srv.poll(t)[0] != 2)
    srv.close()
    lups = sum(r["side"] * r["side"] * r["steps"] for r, _, _, _ in reqs)
    span = reqs[-1][0]["arrival"] if reqs else 0.0
    return dict(requests=len(reqs), warmup_excluded=n_warm, rate_per_s=rate, quantum_steps=quantum,
                hbm_budget_bytes=budget, peak_device_bytes=peak - base,
                p50_s=round(stats["p50_s"], 4), p99_s=round(stats["p99_s"], 4),
                completed_per_s=round(stats["req_per_s"], 2), glups=round(stats["glups"], 2),
                offered_glups=round(lups / max(span, 1e-9) / 1e9, 1), failed=fails,
                offered_glup=round(lups / 1e9, 1), input_generation_s=round(gen_s, 1),
                precision="fp32")


def bench_c2(M, torch, cfg, stream, N):
    """The 2D linear CDE workload (2048^2, MMFD FP32, 10 000 steps) after the
    autotuner, with its step kernel's figures: algorithmic flops against the
    FP32 vector peak, and the committed HBM counters when they match."""
    s32 = c2_solver(M, cfg, "fp32", "mmfd", stream)
    s32.autotune()
    tb, h, w = s32.launch_plan()
    timed(torch, lambda: s32.step(TIME_STEPS))
    ms = timed(torch, lambda: s32.step(TIME_STEPS))
    g = N * TIME_STEPS / (ms * 1e-3) / 1e9
    mean_ms = launch_durations(torch, s32, tb, n=max(1, 4000 // tb)) if tb > 1 else None
    s32.close()
    kname, ksrc = (("k_lane_tb", "kernels_lane_tb.hip") if tb > 1 and w == 128 else
                   ("k_mmfd_tb", "kernels_tb.hip") if tb > 1 else ("k_mmfd_plane", "kernels_mmfd.hip"))
    rec = stored_counters("traffic_mmfd_lcde_d2q9_2048_fp32.json",
                          os.path.join(ROOT, "paper_2505_17057_amd", "csrc", ksrc), tb, w)
    tfl = g * 1e9 * LCDE_D2Q9_FLOPS_PER_LUP / 1e12
    out = dict(glups=round(g, 2), plan=[tb, h, w], kernel=kname, ms_per_solve=round(ms, 3),
               alg_tflops=round(tfl, 2), frac_valu_fp32=round(tfl / VALU_FP32_TFLOPS, 4),
               alg_gbs_depth1=round(g * 8, 1))
    if rec and mean_ms:
        gbs = rec["hbm_bytes_per_launch"] / (mean_ms * 1e-3) / 1e9
        out.update(launch_ms_mean=round(mean_ms, 5), measured_hbm_bytes_per_launch=rec["hbm_bytes_per_launch"],
                   measured_hbm_gbs=round(gbs, 1), measured_hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
                   counters_plan=rec["plan"])
    return out


def headline(M, torch, c3, x0, stream, args):
    """The headline: K full solves of the 4096^2 NSE workload, timed, and the
    roofline figures of its step kernel."""
    log("headline: 4096^2 NSE three-level FP32")
    NH = HEAD_SIDE * HEAD_SIDE
    s32 = _nse_solver(M, "D2Q9", c3, "fp32", stream)
    s32.set_state(x0)
    if args.plan:
        s32.set_plan(*[int(v) for v in args.plan.split(",")])
    else:
        s32.autotune()
    tb, h, w = s32.launch_plan()
    for _ in range(args.warmup):
        timed(torch, lambda: s32.step(HEAD_STEPS))
        s32.reduce()
    # Timed region: K solves, each HEAD_STEPS time steps then the FP64 mass /
    # momentum / residual reduction (each continues from the state the last
    # left); events on the solver's stream split off the step kernels' share
    # to give the mean launch duration.
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    for e0, e1, e2 in ev:
        e0.record()
        s32.step(HEAD_STEPS)
        e1.record()
        s32.reduce()  # synchronous
        e2.record()
    torch.cuda.synchronize()
    ms_per_step = sum(e0.elapsed_time(e2) for e0, _, e2 in ev) / args.steps
    kernel_ms = sum(e0.elapsed_time(e1) for e0, e1, _ in ev) / args.steps
    glups = NH * HEAD_STEPS / (ms_per_step * 1e-3) / 1e9
    if HEAD_STEPS % tb == 0:
        launches = HEAD_STEPS // tb
        mean_ms = kernel_ms / launches
        how = "HIP events on the solver's stream over the timed region: %d launches per solve" % launches
    else:
        mean_ms = launch_durations(torch, s32, tb)
        how = "HIP events on the solver's stream around 1000 back-to-back launches"
    # the step kernel of this plan: the blocked NSE window, or one step a launch
    kname, ksrc = (("k_nse_tb", "kernels_nse_tb.hip") if tb > 1 else
                   ("k_nse_plane_pp", "kernels_mmfd.hip"))
    kernel_src = os.path.join(ROOT, "paper_2505_17057_amd", "csrc", ksrc)
    rec = stored_counters("counters_nse_tb_d2q9_4096_fp32.json", kernel_src, tb, w)
    lups_launch = NH * tb
    alg_flops = NSE_D2Q9_FLOPS_PER_LUP * lups_launch
    achieved = alg_flops / (mean_ms * 1e-3) / 1e12
    traffic = rec["hbm_bytes_per_launch"] if rec else None
    valu = rec["valu_insts_per_launch"] if rec else None
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=round(VALU_FP32_TFLOPS, 2),
                    unit="TFLOP/s", frac=round(achieved / VALU_FP32_TFLOPS, 4), traffic=traffic,
                    kernel=kname + " D2Q9 NSE three-level TRT FP32",
                    kernel_source="paper_2505_17057_amd/csrc/" + ksrc,
                    launch_ms_mean=round(mean_ms, 5), launch_timing=how,
                    time_steps_per_launch=tb, window_rows=h, window_cols=w,
                    algorithmic_flops_per_lup=NSE_D2Q9_FLOPS_PER_LUP,
                    algorithmic_flops_per_launch=alg_flops,
                    peak_derivation="published FP32 vector peak: 256 CUs x 128 lanes x 2 (fused "
                                    "multiply-add) x 2.4 GHz",
                    hbm_algorithmic_bytes_per_lup=36,
                    hbm_algorithmic_gbs_depth1=round(glups * 36, 1),
                    measured_hbm_gbs=(round(traffic / (mean_ms * 1e-3) / 1e9, 1) if traffic else None),
                    measured_hbm_frac=(round(traffic / (mean_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                       if traffic else None),
                    valu_insts_per_launch=valu,
                    valu_insts_per_s=(round(valu / (mean_ms * 1e-3), -6) if valu else None),
                    valu_lane_insts_per_lup=(round(valu * 64 / lups_launch, 1) if valu else None),
                    counters_plan=(rec["plan"] if rec else None))
    s32.close()
    return glups, ms_per_step, tb, roofline



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

    # ---------------------------------------------------------- headline
    c3 = I.tgv_2d(n=HEAD_SIDE)
    NH = HEAD_SIDE * HEAD_SIDE
    x0 = torch.from_numpy(np.ascontiguousarray(c3["state0"], dtype=np.float32)).to("cuda")
    if args.no_headline:
        glups, ms_per_step, tb, roofline = None, None, None, None
    else:
        glups, ms_per_step, tb, roofline = headline(M, torch, c3, x0, stream, args)

    extra = {}
    if args.copy_calibration:
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        extra["copy_calibration_bytes"] = x.numel() * 4  # read once and written once
        del x, y
    sections = set() if args.quick else set(x for x in args.sections.split(",") if x)
    if "c3err" in sections:
        log("headline FP32 error after the full run")
        extra["headline_error"] = bench_c3_error(M, torch, c3, x0, stream)
    del x0
    torch.cuda.empty_cache()
    cfg = I.c2_hill_2d(n=N_SIDE)
    N = N_SIDE * N_SIDE
    if "c2" in sections:
        log("2048^2 linear CDE")
        extra["lcde_d2q9_2048_mmfd_fp32"] = bench_c2(M, torch, cfg, stream, N)
    if "variants" in sections:
        log("variants")
        extra["variants"], extra["fp32_rel_l2_vs_fp64_after_10000"], extra["mesofd_vs_mmfd_fp64_max_abs"] = \
            bench_variants(M, torch, cfg, stream, N)
    if "multiset" in sections:
        log("multiset")
        extra["multiset_d2q9_2048"] = bench_multiset(M, torch, cfg, stream, N)
    if "theta" in sections:
        log("theta")
        extra["theta_d2q9_2048"] = bench_theta(M, torch, cfg, stream, N)
    if "nse_theta" in sections:
        log("NSE theta")
        extra["nse_theta_tgv_1024"] = bench_nse_theta(M, torch, I, stream)
    if "general" in sections:
        log("general scheme")
        extra["general_scheme"] = bench_general(M, torch, I, stream)
    if "rect" in sections:
        log("rectangular lattice")
        extra["rect_lcde_d2q9_2048"] = bench_rect(M, torch, cfg, stream, N)
    if "theta_mg" in sections:
        log("theta, large steps: Jacobi vs multigrid")
        extra["theta_large_dt_d2q9_2048"] = bench_theta_mg(M, torch, cfg, stream, N)
    if "big" in sections:
        log("8192^2")
        extra["hbm_resident_8192_mmfd_fp32"] = bench_big(M, torch, I, stream)
    if "c1" in sections:
        log("1D")
        extra["c1_d1q3_1024"] = bench_c1(M, torch, I, stream)
    if "nse3d" in sections:
        log("NSE 3D")
        extra["nse_d3q19_512_three_level"] = bench_nse3d(M, torch, I, stream, steps=args.nse3d_steps)
    if "source" in sections:
        log("source")
        extra["source_example1_2048"] = bench_source(M, torch, I, stream)
    if "wave" in sections:
        log("wave")
        extra["wave_example3_4096"] = bench_wave(M, torch, stream)
    if "burgers" in sections:
        log("burgers 2048^2")
        extra["burgers_2048_mmfd_fp32"] = bench_burgers_single(M, torch, I, stream)
    if "burgers_theta" in sections:
        log("burgers theta")
        extra["burgers_theta_2048"] = bench_burgers_theta(M, torch, I, stream)
    if "batched" in sections:
        log("batched")
        extra["batched_256_burgers"] = bench_batched(M, torch, I, stream)
        log("batched: small grids")
        extra["batched_512_small_burgers"] = bench_tiny_batch(M, torch, I, stream)
    if "serving" in sections:
        log("serving: requests")
        warm = min(200, args.serve_requests // 10)
        reqs, gen_s, _ = serving_requests(M, I, args.serve_requests, warm=warm)
        log("serving, 200 GB budget")
        extra["serving"] = bench_serving(M, reqs, gen_s, warm)
        log("serving, 2 GB budget")
        extra["serving_2gb_budget"] = bench_serving(M, reqs, gen_s, warm, budget=2 * 10 ** 9)
        del reqs

    cpu = None if args.no_cpu else cpu_baseline(c3)

    line = {
        "metric": "GLUPS + achieved HBM GB/s (% of peak); batched p50/p99 solve latency",
        "value": round(glups, 2) if glups is not None else None,
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4) if ms_per_step is not None else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D incompressible NSE, three-level TRT MMFD, D2Q9, periodic "
                               "4096x4096 Taylor-Green vortex Re = 100 + seeded velocity noise, "
                               "FP32 state with FP64 reductions, 20000 time steps per step",
                   "form": "MMFD", "precision": "fp32 (fp64 reductions)",
                   "time_steps_per_step": HEAD_STEPS, "nodes": NH, "tb_depth": tb},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
