"""GPU: parity at the benchmark's full sizes, in the launch configuration the
benchmark times (autotuned plans), on prefixes of the runs the oracle can
afford, and properties that hold at any size where it cannot.

* 2048^2 linear CDE (the headline workload): FP64 bit-exact with the oracle
  after two blocked launches' worth of steps plus a ragged remainder; FP32
  within 1e-5 (rel. L2) of the oracle; the same at 8192^2.
* 2048^2 MesoFD FP64: populations-carried moments bit-exact with the oracle,
  also under the autotuned blocked plan (FP32 within 1e-5 there).
* 4096^2 NSE three-level TRT: FP64 bit-exact, FP32 within 1e-5.
* 512^3 NSE (D3Q19): mass and momentum conserved by the FP64 step (the
  periodic sum of the central-difference form), FP32 within 1e-6 of FP64.
* 256 Burgers grids: the autotuned blocked batch equals every grid stepped
  alone (FP32, bit for bit), and the smallest grids equal the oracle (FP64).
* 2048^2 three-level Example 1 Case 3 scheme (autotuned): FP64 bit-exact,
  both levels; FP32 within 1e-5.
* 2048^2 Example 1 with its source: FP64 bit-exact, FP32 within 1e-5; the
  MesoFD form FP64 bit-exact (moments and populations).
* 2048^2 theta = 0.5 (4 Jacobi sweeps) and one 2048^2 Burgers grid
  (autotuned): FP64 bit-exact, FP32 within 1e-5.
"""
import numpy as np
import pytest

import mfd_inputs as I
from oracle import native as O
from oracle import scheme as S

pytestmark = pytest.mark.gpu

D0 = 1.0 / 3.0


def _c2_spec(c):
    return dict(lattice="D2Q9", n=c["n"], dx=c["dx"], dt=c["dt"], u=c["u"], K=c["K"], lambda_bar=1,
                a=S.preset_srt()[0])


def _c2_solver(M, c, precision, form="mmfd"):
    s = M.Solver("D2Q9", c["n"], c["dx"], precision, form)
    s.set_equation("lcde", u=c["u"], K=c["K"], lambda_bar=1)
    s.set_scheme("two_level", M.mfd_preset("srt")[0], dt=c["dt"])
    return s


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def c2():
    return I.c2_hill_2d(n=2048)


def test_headline_fp64_bitwise(M, c2):
    steps = 19
    want = c2["phi0"]
    spec = _c2_spec(c2)
    for _ in range(steps):
        want = O.mmfd_step(spec, want)
    s = _c2_solver(M, c2, "fp64")
    s.set_state(c2["phi0"])
    s.autotune()
    print("plan", s.launch_plan(), flush=True)
    s.step(steps)
    got = s.get_state()
    s.close()
    assert np.array_equal(got, want)


def test_headline_fp32_within_tolerance(M, c2):
    steps = 19
    x32 = c2["phi0"].astype(np.float32)
    want = x32.astype(np.float64)
    spec = _c2_spec(c2)
    for _ in range(steps):
        want = O.mmfd_step(spec, want)
    s = _c2_solver(M, c2, "fp32")
    s.set_state(x32)
    s.autotune()
    print("plan", s.launch_plan(), flush=True)
    s.step(steps)
    got = s.get_state().astype(np.float64)
    s.close()
    assert _rel(got, want) <= 1e-5


def test_mesofd_fp64_bitwise(M, c2):
    steps = 3
    spec = _c2_spec(c2)
    pop = O.init_populations(spec, c2["phi0"])
    for _ in range(steps):
        pop, _ = O.mesofd_step(spec, pop, None)
    want = O.moments(spec, pop)
    s = _c2_solver(M, c2, "fp64", "mesofd")
    s.set_state(c2["phi0"])
    s.step(steps)
    assert np.array_equal(s.get_state(), want)
    assert np.array_equal(s.get_state(populations=True), pop)
    s.close()


def _nse(M, lat, c, precision):
    s_ = 1.0 / (c["nu"] / (c["dt"] * D0 * (c["dx"] / c["dt"]) ** 2) + 0.5)
    a, ah = M.mfd_preset("trt", s_)
    s = M.Solver(lat, c["n"], c["dx"], precision, "mmfd")
    s.set_equation("nse", rho0=c["rho0"])
    s.set_scheme("three_level", a, ah, dt=c["dt"])
    spec = dict(lattice=lat, eq="nse", n=c["n"], dx=c["dx"], dt=c["dt"], rho0=c["rho0"], a=a, ah=ah,
                levels=3)
    return s, spec


def test_nse_2d_4096(M):
    c = I.tgv_2d(n=4096)
    x32 = c["state0"].astype(np.float32)
    x = x32.astype(np.float64)
    s, spec = _nse(M, "D2Q9", c, "fp64")
    steps = 2
    cur, prev = x, x
    for _ in range(steps):
        cur, prev = O.mmfd_step(spec, cur, prev), cur
    s.set_state(x)
    s.step(steps)
    assert np.array_equal(s.get_state(), cur)
    assert np.array_equal(s.get_state(level=1), prev)
    s.close()
    s32, _ = _nse(M, "D2Q9", c, "fp32")
    s32.set_state(x32)
    s32.step(steps)
    assert _rel(s32.get_state().astype(np.float64), cur) <= 1e-5
    s32.close()


def test_nse_3d_512_conservation(M):
    import torch
    c = I.tgv_3d(n=512, dtype=np.float32)
    x32 = torch.from_numpy(c["state0"]).to("cuda")
    del c["state0"]
    N = 512 ** 3
    s64, _ = _nse(M, "D3Q19", c, "fp64")
    x64 = x32.double()
    s64.set_state(x64)
    sums0, _ = s64.reduce()
    s64.step(2)
    sums2, _ = s64.reduce()
    y64 = torch.empty_like(x64)
    s64.get_state(out=y64)
    s64.close()
    for f in range(4):
        scale = float(x64[f * N:(f + 1) * N].abs().sum())
        assert abs(sums2[f] - sums0[f]) <= 1e-12 * scale, (f, sums0[f], sums2[f])
    s32, _ = _nse(M, "D3Q19", c, "fp32")
    s32.set_state(x32)
    s32.step(2)
    y32 = torch.empty_like(x32)
    s32.get_state(out=y32)
    s32.close()
    torch.cuda.synchronize()
    err = float(torch.linalg.vector_norm(y32.double() - y64) / torch.linalg.vector_norm(y64))
    assert err <= 1e-6, err


def _burgers(M, c, precision):
    s = M.Solver("D2Q9", c["n"], c["dx"], precision, "mmfd")
    s.set_equation("burgers")
    sp = 2 * c["nu"] * c["dt"] / (D0 * c["dx"] ** 2)
    a = ((sp + 1) / 2, 1 - sp, (sp - 1) / 2)
    s.set_scheme("two_level", a, dt=c["dt"])
    return s, a


def test_batched_256_burgers(M):
    insts = I.c4_batch(256, seed=4)
    steps = [min(c["steps"], 13 + (i % 7)) for i, c in enumerate(insts)]  # ragged prefixes
    solo = []
    for c, n in zip(insts, steps):
        s, _ = _burgers(M, c, "fp32")
        s.set_blocking(1)
        s.set_state(c["phi0"].astype(np.float32))
        s.step(n)
        solo.append(s.get_state())
        s.close()
    b = M.Batch()
    solvers = []
    for c, n in zip(insts, steps):
        s, _ = _burgers(M, c, "fp32")
        s.set_state(c["phi0"].astype(np.float32))
        b.add(s, n)
        solvers.append(s)
    b.autotune()
    b.run()
    b.wait()
    print("plan", b.plan(0), flush=True)
    for i, (s, want) in enumerate(zip(solvers, solo)):
        assert np.array_equal(s.get_state(), want), i
    b.close()
    for s in solvers:
        s.close()
    # FP64 batch against the oracle on the four smallest grids
    small = sorted(range(256), key=lambda i: insts[i]["n"][0])[:4]
    b = M.Batch()
    b.set_plan(4, 48)
    keep = []
    for i in small:
        c = insts[i]
        s, a = _burgers(M, c, "fp64")
        s.set_state(c["phi0"])
        b.add(s, steps[i])
        keep.append((i, s, a))
    b.run()
    b.wait()
    for i, s, a in keep:
        c = insts[i]
        spec = dict(lattice="D2Q9", eq="burgers", n=c["n"], dx=c["dx"], dt=c["dt"], a=a)
        want = c["phi0"]
        for _ in range(steps[i]):
            want = O.mmfd_step(spec, want)
        assert np.array_equal(s.get_state(), want), i
        s.close()
    b.close()


def _three_level_c2(M, c, precision):
    s = M.Solver("D2Q9", c["n"], c["dx"], precision, "mmfd")
    s.set_equation("lcde", u=c["u"], K=c["K"], lambda_bar=1)
    s.set_scheme("three_level", (7 / 8, 0.0, 1 / 8), (1 / 8, 0.0, -1 / 8), dt=c["dt"])
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_three_level_case3(M, c2, precision):
    """The three-level scheme of Example 1 Case 3 on the 2048^2 workload, both
    levels starting from phi0, autotuned plan: FP64 bit-exact with the oracle,
    FP32 within 1e-5 (rel. L2)."""
    steps = 13
    x0 = c2["phi0"].astype(np.float32 if precision == "fp32" else np.float64)
    spec = dict(_c2_spec(c2), a=(7 / 8, 0.0, 1 / 8), ah=(1 / 8, 0.0, -1 / 8), levels=3)
    cur, prev = x0.astype(np.float64), x0.astype(np.float64)
    for _ in range(steps):
        cur, prev = O.mmfd_step(spec, cur, prev), cur
    s = _three_level_c2(M, c2, precision)
    s.set_state(x0)
    s.set_state(x0, level=1)
    s.autotune()
    print("plan", s.launch_plan(), flush=True)
    s.step(steps)
    got, got_prev = s.get_state().astype(np.float64), s.get_state(level=1).astype(np.float64)
    s.close()
    if precision == "fp64":
        assert np.array_equal(got, cur) and np.array_equal(got_prev, prev)
    else:
        assert _rel(got, cur) <= 1e-5 and _rel(got_prev, prev) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_source_example1_2048(M, precision):
    """Example 1 with its source (three-level Case 2, b_-1 = 3/2, bh_-1 = -1/2)
    on the 2048^2 grid the benchmark times: FP64 bit-exact with the oracle
    over 6 steps in two calls, FP32 within 1e-5."""
    import math
    ex = I.example1_source_2d(n=2048)
    a, ah = (7 / 8, 1 / 4, -1 / 8), (1 / 8, -1 / 4, 1 / 8)
    coef = dict(b=(1.5, 0.0, 0.0), bh=(-0.5, 0.0, 0.0))
    spec = dict(lattice="D2Q9", eq="lcde", n=ex["n"], dx=ex["dx"], dt=ex["dt"], u=ex["u"], K=ex["K"],
                lambda_bar=1, a=a, ah=ah, levels=3)
    dt, lam, G = ex["dt"], ex["lam"], ex["G"]
    ftype = np.float32 if precision == "fp32" else np.float64
    cur, prev = ex["phi0"].astype(ftype).astype(np.float64), ex["phim"].astype(ftype).astype(np.float64)
    for k in range(6):
        src = dict(coef, v=ex["u"], S_t=math.exp(lam * (k * dt)) * G,
                   S_m=math.exp(lam * ((k - 1) * dt)) * G)
        cur, prev = O.mmfd_step(spec, cur, prev, src), cur
    s = M.Solver("D2Q9", ex["n"], ex["dx"], precision, "mmfd")
    s.set_equation("lcde", u=ex["u"], K=ex["K"], lambda_bar=1)
    s.set_scheme("three_level", a, ah, dt=dt)
    s.set_state(ex["phi0"].astype(ftype))
    s.set_state(ex["phim"].astype(ftype), level=1)
    s.set_source(G, lam, coef["b"], coef["bh"], ex["u"])
    s.step(4)
    s.step(2)
    got = s.get_state().astype(np.float64)
    s.close()
    if precision == "fp64":
        assert np.array_equal(got, cur)
    else:
        assert _rel(got, cur) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_theta_2048(M, c2, precision):
    """The theta = 0.5 scheme with 4 Jacobi sweeps per step on the 2048^2
    workload: FP64 bit-exact with the oracle over 5 steps, FP32 within 1e-5."""
    steps = 5
    spec = dict(_c2_spec(c2), theta=0.5, theta_iters=4)
    x0 = c2["phi0"].astype(np.float32 if precision == "fp32" else np.float64)
    want = x0.astype(np.float64)
    for _ in range(steps):
        want = O.theta_step(spec, want)
    s = M.Solver("D2Q9", c2["n"], c2["dx"], precision, "mmfd")
    s.set_equation("lcde", u=c2["u"], K=c2["K"], lambda_bar=1)
    s.set_scheme("theta", M.mfd_preset("srt")[0], theta=0.5, theta_iters=4, dt=c2["dt"])
    s.set_state(x0)
    s.step(steps)
    got = s.get_state().astype(np.float64)
    s.close()
    if precision == "fp64":
        assert np.array_equal(got, want)
    else:
        assert _rel(got, want) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_burgers_2048(M, precision):
    """One 2048^2 Burgers grid of the batched workload's recipe, autotuned plan:
    FP64 bit-exact with the oracle over 25 steps, FP32 within 1e-5."""
    rng = np.random.default_rng(6)
    c = I.burgers_instance(rng, side_lo=2048, side_hi=2048, steps_lo=1000, steps_hi=1000)
    a = M.mfd_preset("two_level", 2.0 * c["nu"] * c["dt"] / (D0 * c["dx"] ** 2))[0]
    spec = dict(lattice="D2Q9", eq="burgers", n=c["n"], dx=c["dx"], dt=c["dt"], a=a, levels=2,
                ah=(0.0, 0.0, 0.0))
    steps = 25
    x0 = c["phi0"].astype(np.float32 if precision == "fp32" else np.float64)
    want = x0.astype(np.float64)
    for _ in range(steps):
        want = O.mmfd_step(spec, want)
    s = M.Solver("D2Q9", c["n"], c["dx"], precision, "mmfd")
    s.set_equation("burgers")
    s.set_scheme("two_level", a, dt=c["dt"])
    s.set_state(x0)
    s.autotune()
    print("plan", s.launch_plan(), flush=True)
    s.step(steps)
    got = s.get_state().astype(np.float64)
    s.close()
    if precision == "fp64":
        assert np.array_equal(got, want)
    else:
        assert _rel(got, want) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mesofd_autotuned_2048(M, c2, precision):
    """MesoFD on the 2048^2 workload under the autotuned blocked plan the
    benchmark times, 23 steps (two blocked launches and a ragged remainder at
    the usual depths): FP64 moments and populations bit-exact with the
    oracle, FP32 moments within 1e-5."""
    steps = 23
    spec = _c2_spec(c2)
    x0 = c2["phi0"].astype(np.float32 if precision == "fp32" else np.float64)
    pop = O.init_populations(spec, x0.astype(np.float64))
    for _ in range(steps):
        pop, _ = O.mesofd_step(spec, pop, None)
    want = O.moments(spec, pop)
    s = _c2_solver(M, c2, precision, "mesofd")
    s.set_state(x0)
    s.autotune()
    print("plan", s.launch_plan(), flush=True)
    s.step(steps)
    got = s.get_state().astype(np.float64)
    if precision == "fp64":
        assert np.array_equal(got, want)
        assert np.array_equal(s.get_state(populations=True), pop)
    else:
        assert _rel(got, want) <= 1e-5
    s.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_headline_8192(M, precision):
    """The 8192^2 grid of the same workload under its autotuned plan, 27 steps
    (two blocked launches at depth 12 and a ragged remainder): FP32 within
    1e-5 of the oracle, FP64 bit-exact."""
    big = I.c2_hill_2d(n=8192)
    steps = 27
    x0 = big["phi0"].astype(np.float32 if precision == "fp32" else np.float64)
    want = x0.astype(np.float64)
    spec = _c2_spec(big)
    for _ in range(steps):
        want = O.mmfd_step(spec, want)
    s = _c2_solver(M, big, precision)
    s.set_state(x0)
    s.autotune()
    print("plan", s.launch_plan(), flush=True)
    s.step(steps)
    got = s.get_state().astype(np.float64)
    s.close()
    if precision == "fp64":
        assert np.array_equal(got, want)
    else:
        assert _rel(got, want) <= 1e-5


def test_source_example1_mesofd_2048(M):
    """The MesoFD form of the Example 1 step with its source on the 2048^2
    grid the benchmark times: FP64 moments and populations bit-exact with the
    oracle over 4 steps in two calls."""
    import math
    ex = I.example1_source_2d(n=2048)
    a, ah = (7 / 8, 1 / 4, -1 / 8), (1 / 8, -1 / 4, 1 / 8)
    coef = dict(b=(1.5, 0.0, 0.0), bh=(-0.5, 0.0, 0.0))
    spec = dict(lattice="D2Q9", eq="lcde", n=ex["n"], dx=ex["dx"], dt=ex["dt"], u=ex["u"], K=ex["K"],
                lambda_bar=1, a=a, ah=ah, levels=3)
    pop, pm = O.init_populations(spec, ex["phi0"]), ex["phim"]
    for k in range(4):
        src = dict(coef, v=ex["u"], S_t=math.exp(ex["lam"] * (k * ex["dt"])) * ex["G"],
                   S_m=math.exp(ex["lam"] * ((k - 1) * ex["dt"])) * ex["G"])
        pop, pm = O.mesofd_step(spec, pop, pm, src)
    want = O.moments(spec, pop)
    s = M.Solver("D2Q9", ex["n"], ex["dx"], "fp64", "mesofd")
    s.set_equation("lcde", u=ex["u"], K=ex["K"], lambda_bar=1)
    s.set_scheme("three_level", a, ah, dt=ex["dt"])
    s.set_state(ex["phi0"])
    s.set_state(ex["phim"], level=1)
    s.set_source(ex["G"], ex["lam"], coef["b"], coef["bh"], ex["u"])
    s.step(1)
    s.step(3)
    got, gpop = s.get_state(), s.get_state(populations=True)
    s.close()
    assert np.array_equal(got, want)
    assert np.array_equal(gpop, pop)
