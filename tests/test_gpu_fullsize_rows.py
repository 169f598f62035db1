"""GPU: parity at the benchmark's sizes for the rows beyond the headline
workloads, in the configurations the benchmark times.

* NSE theta = 0.5 on the 1024^2 Taylor-Green vortex (dt = 0.2 dx / U0,
  density set s = 1, momentum set s from nu), each step solved to 1e-12:
  FP64 bit-exact with the oracle's Picard iteration over two steps, sweep
  counts equal; FP32 (to 1e-6) within 1e-5.
* The general-scheme solver: rD3Q27 linear CDE at 256^3 (reach 1), the
  2048^2 rD2Q9 linear CDE with reach 2 and two levels, the 1024^2 rD2Q9 NSE
  with reach 2: FP64 bit-exact with the oracle's central form, FP32 within
  1e-5.
* The 2048^2 rectangular rD2Q9 linear CDE (dy = 2 dx, d0 = (1/3, 1/4)) under
  the autotuned plan: FP64 bit-exact with the oracle after two launches and a
  ragged remainder, FP32 within 1e-5.
"""
import numpy as np
import pytest

import mfd_inputs as I
from oracle import general as GN
from parity_util import make_solver, oracle_spec, rel_l2, run_oracle

pytestmark = pytest.mark.gpu

D0 = 1.0 / 3.0


def _fam(s):
    return ((s + 1) / 2, 1 - s, (s - 1) / 2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nse_theta_tgv_1024(M, precision):
    from oracle import implicit as IM

    c = I.tgv_2d(n=1024, courant=0.2)
    s_j = 1.0 / (c["nu"] * c["dt"] / (D0 * c["dx"] ** 2) + 0.5)
    case = dict(lattice="D2Q9", n=c["n"], dx=c["dx"], dt=c["dt"], eq="nse", rho0=c["rho0"],
                a=_fam(1.0), ab=_fam(s_j), kind="theta", theta=0.5, theta_iters=64)
    spec = oracle_spec(case)
    dt = np.float64 if precision == "fp64" else np.float32
    x = c["state0"].astype(dt)
    want, sweeps = x.astype(np.float64), []
    for _ in range(2):
        want, k, conv = IM.theta_picard_solve(spec, want, 1e-12, 4, 64)
        assert conv
        sweeps.append(k)
    s = make_solver(M, case, precision)
    s.set_theta_tolerance(1e-12 if precision == "fp64" else 1e-6, 4)
    s.set_state(x)
    s.step(2)
    got = s.get_state().astype(np.float64)
    st = s.theta_stats()
    s.close()
    assert st["unconverged"] == 0
    if precision == "fp64":
        assert st["total_sweeps"] == sum(sweeps)
        assert np.array_equal(got, want)
    else:
        assert rel_l2(got, want) < 1e-5


ONE = np.array([[1.0, 0.0, 0.0]])
TWO = np.array([[0.2, 0.6, 0.2, 0.0, 0.0], [-0.05, 0.1, -0.05, 0.0, 0.0]])
WIDE = np.array([[0.25, 0.5, 0.25, 0.0, 0.0]])
GEN = [
    dict(name="lcde-d3q27-256-m1", lattice="D3Q27", n=(256, 256, 256), a=ONE, steps=1),
    dict(name="lcde-d2q9-2048-m2-n2", lattice="D2Q9", n=(2048, 2048), a=TWO, steps=3),
    dict(name="nse-d2q9-1024-m2", lattice="D2Q9", n=(1024, 1024), a=WIDE, steps=2, eq="nse"),
]


def _gen_inputs(c):
    n, dim = c["n"], len(c["n"])
    if c.get("eq") == "nse":
        t = I.tgv_2d(n=n[0])
        spec = dict(lattice=c["lattice"], eq="nse", n=n, dx=t["dx"], dt=t["dt"], rho0=t["rho0"],
                    beta=1.0)
        return spec, t["state0"]
    x = np.indices(tuple(reversed(n)), dtype=np.float64)
    state = np.exp(sum(np.cos(2 * np.pi * x[i] / n[dim - 1 - i]) for i in range(dim))).ravel()
    spec = dict(lattice=c["lattice"], eq="lcde", n=n, dx=1.0, dt=1.0, u=[0.05, -0.03, 0.02][:dim],
                K=(np.eye(dim) * 0.1).tolist(), lambda_bar=1)
    return spec, state


def _gen_gpu(M, c, spec, state, precision):
    a = c["a"]
    if spec["eq"] == "nse":
        g = M.General(c["lattice"], c["n"], spec["dx"], a, spec["dt"], precision=precision,
                      eq="nse", ab=a, rho0=spec["rho0"])
    else:
        g = M.General(c["lattice"], c["n"], 1.0, a, 1.0, u=spec["u"], K=spec["K"], lambda_bar=1,
                      precision=precision)
    g.set_level(0, state)
    g.step(c["steps"])
    out = g.get_level(0).astype(np.float64)
    g.close()
    return out


def _gen_oracle(c, spec, state):
    a = c["a"]
    lev = [np.asarray(state, dtype=np.float64)] * a.shape[0]
    for _ in range(c["steps"]):
        if spec["eq"] == "nse":
            new = GN.nonlinear_mmfd_step(spec, lev, a, a)
        else:
            new = GN.mmfd_step(spec, lev, a)
        lev = [new] + lev[:-1]
    return lev[0]


@pytest.mark.parametrize("case", GEN, ids=lambda c: c["name"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_general_benchmark_sizes(M, case, precision):
    spec, state = _gen_inputs(case)
    if precision == "fp32":
        state = state.astype(np.float32).astype(np.float64)
    want = _gen_oracle(case, spec, state)
    got = _gen_gpu(M, case, spec, state, precision)
    if precision == "fp64":
        assert np.array_equal(got, want)
    else:
        assert rel_l2(got, want) < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rect_2048_autotuned(M, precision):
    cfg = I.c2_hill_2d(n=2048)
    case = dict(lattice="D2Q9", n=cfg["n"], dx=cfg["dx"], dt=cfg["dt"], u=cfg["u"], K=cfg["K"],
                lambda_bar=1, a=(1.0, 0.0, 0.0), dxv=(cfg["dx"], 2 * cfg["dx"]),
                d0v=(D0, 0.25))
    dt = np.float64 if precision == "fp64" else np.float32
    phi = cfg["phi0"].astype(dt)
    s = make_solver(M, case, precision)
    s.set_state(phi)
    s.autotune()
    tb = s.launch_plan()[0]
    steps = 2 * tb + 3
    s.set_state(phi)
    s.step(steps)
    got = s.get_state().astype(np.float64)
    s.close()
    want = run_oracle(case, phi.astype(np.float64), None, steps)
    if precision == "fp64":
        assert np.array_equal(got, want)
    else:
        assert rel_l2(got, want) < 1e-5
