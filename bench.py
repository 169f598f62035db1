"""Benchmark of the MesoFD / MMFD time step on one MI355X.

Headline workload (the one the metric is quoted on): 2D anisotropic linear
CDE, D2Q9, periodic 2048 x 2048, K = [[0.02,0.005],[0.005,0.01]],
u = (0.05, 0.03), dt = 2^-18, SRT coefficients, Gaussian hill + seeded noise,
10 000 time steps per solve.  One benchmark "step" is one full solve
(10 000 time steps of the MMFD form in FP32, then an FP64 mass reduction).

Beside it the same JSON line reports
* the other forms / precisions of that workload and an HBM-resident 8192^2 point,
* the FP32 error of the full run against the FP64 run,
* the 1D D1Q3 workload (1024 nodes, 1000 steps, LDS-resident),
* the NSE three-level MMFD workloads (4096^2 D2Q9, 512^3 D3Q19),
* the batched workload: 256 Burgers grids, one graph launch in FP32, against
  plain per-instance FP64 stepping,
* the serving workload: Poisson arrivals of mixed Burgers / NSE solves,
  p50 / p99 latency and throughput,
* the oracle on the host cores (CPU baseline).

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
TIME_STEPS = 10000
N_SIDE = 2048
D0 = 1.0 / 3.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--quick", action="store_true", help="headline only (for profiling)")
    p.add_argument("--sections", default="variants,theta,big,c1,nse,source,burgers,batched,serving",
                   help="comma-separated sections to run after the headline")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a 256 MiB device copy (HBM counter calibration)")
    p.add_argument("--serve-requests", type=int, default=300)
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


def stored_traffic(kernel_src, tb, h, w):
    """(HBM bytes per launch, profiled plan) from the committed rocprofv3
    counter summary, if it was taken on the current kernel source with the
    same steps per launch and window width (the window height changes only
    halo re-reads, which the profiled plan states); else (None, None)."""
    path = os.path.join(ROOT, "profiles", "traffic_mmfd_lcde_d2q9_2048_fp32.json")
    if not os.path.exists(path):
        return None, None
    info = json.load(open(path))
    sha = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if info.get("kernel_source_sha256") != sha:
        return None, None
    for r in [info] + info.get("alternates", []):
        if r.get("time_steps_per_launch") == tb and r.get("window_cols") == w:
            plan = [r.get("time_steps_per_launch"), r.get("window_rows"), r.get("window_cols")]
            return r.get("hbm_bytes_per_launch"), plan
    return None, None


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
    return dict(value=round(N * steps / el / 1e9, 4), unit="GLUPS", cores=threads, kind="oracle",
                sample="%d MMFD FP64 time steps of the 2048^2 D2Q9 linear-CDE workload (%.1f s)"
                       % (steps, el))


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


def bench_theta(M, torch, cfg, stream, N, theta=0.5, sweeps=4, steps=1000):
    """theta scheme (linear CDE) on the headline grid: right-hand side plus
    `sweeps` Jacobi sweeps per time step, FP32, and its error against the
    FP64 run of the same steps."""
    out = {}
    finals = {}
    for prec in ("fp32", "fp64"):
        s = M.Solver("D2Q9", cfg["n"], cfg["dx"], prec, "mmfd")
        s.set_equation("lcde", u=cfg["u"], K=cfg["K"], lambda_bar=cfg["lambda_bar"])
        s.set_scheme("theta", M.mfd_preset("srt")[0], theta=theta, theta_iters=sweeps, dt=cfg["dt"])
        s.set_stream(stream.cuda_stream)
        s.set_state(cfg["phi0"].astype(s.dtype))
        s.step(10)
        s.set_state(cfg["phi0"].astype(s.dtype))
        ms = timed(torch, lambda: s.step(steps))
        finals[prec] = s.get_state().astype(np.float64)
        s.close()
        g = N * steps / (ms * 1e-3) / 1e9
        bpl = (2 + 3 * sweeps) * (4 if prec == "fp32" else 8)  # rhs: read + write; sweep: 2 reads + write
        out[prec] = dict(glups=round(g, 2), alg_gbs=round(g * bpl, 1), frac_hbm=round(g * bpl / HBM_PEAK_GBS, 4),
                         bytes_per_lup=bpl)
    out.update(theta=theta, jacobi_sweeps=sweeps, steps=steps,
               fp32_rel_l2_vs_fp64=float(np.linalg.norm(finals["fp32"] - finals["fp64"])
                                         / np.linalg.norm(finals["fp64"])))
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
    res = {}
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
        s.step(20)
        start()
        ms = timed(torch, lambda: s.step(steps))
        finals[prec, form] = s.get_state().astype(np.float64)
        s.close()
        g = ex["n"][0] * ex["n"][1] * steps / (ms * 1e-3) / 1e9
        es = 8 if prec == "fp64" else 4
        key = prec if form == "mmfd" else "mesofd_" + prec
        if form == "mmfd":
            bpl = 4 * es  # read t, t - dt and G; write t + dt
            out[key] = dict(glups=round(g, 2), alg_gbs=round(g * bpl, 1),
                            frac_hbm=round(g * bpl / HBM_PEAK_GBS, 4), bytes_per_lup=bpl)
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


def bench_nse(M, torch, I, stream):
    """Three-level TRT NSE: FP32 timing, and the FP32 error against the FP64
    run of the same steps from the same (binary32-rounded) start."""
    res = {}
    for lat, c, warm, steps, bpl, key in (
            ("D2Q9", I.tgv_2d(n=4096), 20, 200, 36, "d2q9_4096_three_level_fp32"),
            ("D3Q19", I.tgv_3d(n=512, dtype=np.float32), 2, 20, 48, "d3q19_512_three_level_fp32")):
        x0 = torch.from_numpy(np.ascontiguousarray(c["state0"], dtype=np.float32)).to("cuda")
        del c["state0"]
        nodes = int(np.prod(c["n"]))
        s = _nse_solver(M, lat, c, "fp32", stream)
        s.set_state(x0)
        s.autotune()
        plan = s.launch_plan()
        s.step(warm)
        ms = timed(torch, lambda: s.step(steps))
        g = nodes * steps / (ms * 1e-3) / 1e9
        y32 = torch.empty_like(x0)
        s.get_state(out=y32)
        s.close()
        s64 = _nse_solver(M, lat, c, "fp64", stream)
        x64 = x0.double()
        s64.set_state(x64)
        s64.step(warm + steps)
        y64 = torch.empty_like(x64)
        s64.get_state(out=y64)
        s64.close()
        torch.cuda.synchronize()
        res[key] = dict(glups=round(g, 2), alg_gbs=round(g * bpl, 1),
                        frac_hbm=round(g * bpl / HBM_PEAK_GBS, 4), bytes_per_lup=bpl,
                        steps=warm + steps, plan=list(plan),
                        fp32_rel_l2_vs_fp64=_rel_l2_dev(torch, y32, y64))
        del x0, x64, y32, y64
        torch.cuda.empty_cache()
    return res


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


def bench_serving(M, I, n_total, rate=200.0, warm=50, quantum=50):
    trace = I.serving_trace(count=n_total - warm, warmup=warm, rate=rate)
    reqs = []
    t0 = time.perf_counter()
    for r in trace:
        inst = I.serving_request_state(r)
        dx, dt = inst["dx"], inst["dt"]
        if r["kind"] == "burgers":
            st = inst["phi0"].astype(np.float32)
            a, ah, kind, eq, rho0 = two_level_a(M, inst["nu"], dx, dt), None, "two_level", "burgers", 0.0
        else:
            st = inst["state0"].astype(np.float32)
            a, ah = trt_coeffs(M, inst["nu"], dx, dt)
            kind, eq, rho0 = "three_level", "nse", inst["rho0"]
        out = np.empty_like(st)
        req = M.make_request("D2Q9", eq, inst["n"], dx, dt, a, r["steps"], st, ah=ah, kind=kind,
                             precision="fp32", rho0=rho0, result_out=out, exclude=r["warmup"])
        reqs.append((r, req, st, out))
    gen_s = time.perf_counter() - t0
    srv = M.Server(hbm_budget_bytes=200 * 10 ** 9, max_slots=1024, quantum_steps=quantum)
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
    stats = srv.stats()
    fails = sum(1 for t in tickets if srv.poll(t)[0] != 2)
    srv.close()
    lups = sum(r["side"] * r["side"] * r["steps"] for r, _, _, _ in reqs)
    return dict(requests=len(reqs), warmup_excluded=warm, rate_per_s=rate, quantum_steps=quantum,
                hbm_budget_bytes=200 * 10 ** 9, p50_s=round(stats["p50_s"], 4),
                p99_s=round(stats["p99_s"], 4), completed_per_s=round(stats["req_per_s"], 2),
                glups=round(stats["glups"], 2), failed=fails, offered_glup=round(lups / 1e9, 1),
                input_generation_s=round(gen_s, 1), precision="fp32")


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
    log("headline: 2048^2 MMFD FP32")
    s32 = c2_solver(M, cfg, "fp32", "mmfd", stream)
    if args.plan:
        s32.set_plan(*[int(v) for v in args.plan.split(",")])
    else:
        s32.autotune()
    tb, h, w = s32.launch_plan()
    for _ in range(args.warmup):
        timed(torch, lambda: s32.step(TIME_STEPS))
        s32.reduce()
    # Timed region: K solves, each TIME_STEPS time steps then the FP64 mass /
    # residual reduction; events on the solver's stream split off the step
    # kernels' share to give the mean launch duration.
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    for e0, e1, e2 in ev:
        e0.record()
        s32.step(TIME_STEPS)
        e1.record()
        s32.reduce()  # synchronous
        e2.record()
    torch.cuda.synchronize()
    ms_per_step = sum(e0.elapsed_time(e2) for e0, _, e2 in ev) / args.steps
    kernel_ms = sum(e0.elapsed_time(e1) for e0, e1, _ in ev) / args.steps
    glups = N * TIME_STEPS / (ms_per_step * 1e-3) / 1e9
    if TIME_STEPS % tb == 0:
        launches = TIME_STEPS // tb
        mean_ms = kernel_ms / launches
        how = "HIP events over the timed region: %d launches per solve" % launches
    else:
        mean_ms = launch_durations(torch, s32, tb)
        how = "HIP events around 1000 back-to-back launches"
    alg_bytes = 8.0 * N * tb  # read phi^n, write phi^(n+1): 8 B per LUP in FP32
    achieved = alg_bytes / (mean_ms * 1e-3) / 1e9
    # the step kernel of this plan: the in-place lane-shared LCDE window (128
    # columns), the general blocked window (64 columns), or one step a launch
    kname, ksrc = (("k_lane_tb", "kernels_lane_tb.hip") if tb > 1 and w == 128 else
                   ("k_mmfd_tb", "kernels_tb.hip") if tb > 1 else
                   ("k_mmfd_plane", "kernels_mmfd.hip"))
    kernel_src = os.path.join(ROOT, "paper_2505_17057_amd", "csrc", ksrc)
    traffic, traffic_plan = stored_traffic(kernel_src, tb, h, w)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel=kname + " D2Q9 LCDE FP32",
                    kernel_source="paper_2505_17057_amd/csrc/" + ksrc,
                    launch_ms_mean=round(mean_ms, 5), launch_timing=how,
                    time_steps_per_launch=tb, window_rows=h, window_cols=w,
                    algorithmic_bytes_per_launch=alg_bytes,
                    measured_hbm_gbs=(round(traffic / (mean_ms * 1e-3) / 1e9, 1) if traffic else None),
                    traffic_plan=traffic_plan)
    s32.close()

    extra = {}
    if args.copy_calibration:
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        extra["copy_calibration_bytes"] = x.numel() * 4  # read once and written once
    sections = set() if args.quick else set(x for x in args.sections.split(",") if x)
    if "variants" in sections:
        log("variants")
        extra["variants"], extra["fp32_rel_l2_vs_fp64_after_10000"], extra["mesofd_vs_mmfd_fp64_max_abs"] = \
            bench_variants(M, torch, cfg, stream, N)
    if "theta" in sections:
        log("theta")
        extra["theta_d2q9_2048"] = bench_theta(M, torch, cfg, stream, N)
    if "big" in sections:
        log("8192^2")
        extra["hbm_resident_8192_mmfd_fp32"] = bench_big(M, torch, I, stream)
    if "c1" in sections:
        log("1D")
        extra["c1_d1q3_1024"] = bench_c1(M, torch, I, stream)
    if "nse" in sections:
        log("NSE")
        extra["nse"] = bench_nse(M, torch, I, stream)
    if "source" in sections:
        log("source")
        extra["source_example1_2048"] = bench_source(M, torch, I, stream)
    if "burgers" in sections:
        log("burgers 2048^2")
        extra["burgers_2048_mmfd_fp32"] = bench_burgers_single(M, torch, I, stream)
    if "batched" in sections:
        log("batched")
        extra["batched_256_burgers"] = bench_batched(M, torch, I, stream)
    if "serving" in sections:
        log("serving")
        extra["serving"] = bench_serving(M, I, args.serve_requests)

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
    print(json.dumps(line))


if __name__ == "__main__":
    main()
