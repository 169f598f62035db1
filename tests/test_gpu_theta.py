"""GPU: the theta scheme of Eq. (GCN) solved to a residual tolerance.

Each case runs several time steps on the GPU and the same steps with the
oracle's to-tolerance solve (orc_theta_solve: the same chunked stopping rule
in binary64 with compensated sums):
* binary64: every state bit-exact, and the sweeps the GPU reports equal the
  oracle's (the decision could only differ where the residual ratio sits
  within round-off of the tolerance, which the test detects and reports);
* binary32 at 1e-6: relative L2 within 1e-5 of the oracle's binary64 solve.
The device-decided path (2D windows) and the host-checked path (small, 1D and
3D grids) are both covered, as are ragged tiles and a stop forced by the cap.
"""
import numpy as np
import pytest

from oracle import native as O
from parity_util import make_solver, oracle_spec, rel_l2

pytestmark = pytest.mark.gpu

K2 = [[0.3, 0.04], [0.04, 0.2]]

CASES = [
    dict(name="d2q9-fused", lattice="D2Q9", n=(203, 150), u=(0.1, -0.07), K=K2, lambda_bar=1),
    dict(name="d2q5-fused", lattice="D2Q5", n=(130, 77), u=(0.05, 0.02), K=[[0.2, 0.0], [0.0, 0.2]]),
    dict(name="d2q9-small", lattice="D2Q9", n=(40, 21), u=(0.1, -0.07), K=K2, lambda_bar=1),
    dict(name="d1q3", lattice="D1Q3", n=(300,), u=(0.1,), K=[[0.3]]),
    dict(name="d3q19", lattice="D3Q19", n=(14, 11, 9), u=(0.05, 0.02, -0.03),
         K=[[0.1, 0, 0], [0, 0.1, 0], [0, 0, 0.1]]),
]


def _case(c, cap):
    a = (1.0, 0.0, 0.0)  # SRT tau = 1 (a_-1 = 1)
    return dict(c, eq="lcde", a=a, kind="theta", theta=0.5, theta_iters=cap, dx=1.0, dt=1.0)


def _oracle_run(case, phi, steps, tol, chunk, cap):
    spec = oracle_spec(case)
    sweeps = []
    for _ in range(steps):
        phi, k, _ = O.theta_solve(spec, phi, tol, chunk, cap)
        sweeps.append(k)
    return phi, sweeps


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
@pytest.mark.parametrize("tol,chunk", [(1e-12, 8), (1e-9, 3)])
def test_theta_tolerance_fp64_matches_oracle(M, case, tol, chunk):
    cap, steps = 96, 4
    c = _case(case, cap)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal(int(np.prod(c["n"])))
    want, sweeps = _oracle_run(c, phi, steps, tol, chunk, cap)
    s = make_solver(M, c, "fp64")
    s.set_theta_tolerance(tol, chunk)
    s.set_state(phi)
    s.step(1)
    s.step(steps - 1)
    got = s.get_state()
    st = s.theta_stats()
    s.close()
    assert st["steps"] == steps and st["unconverged"] == 0
    assert st["total_sweeps"] == sum(sweeps), (st, sweeps)
    assert st["max_sweeps"] == max(sweeps)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("case", [CASES[0], CASES[2]], ids=["fused", "host-checked"])
def test_theta_tolerance_fp32_within_1e5(M, case):
    cap, steps = 96, 6
    c = _case(case, cap)
    rng = np.random.default_rng(6)
    phi = rng.standard_normal(int(np.prod(c["n"])))
    phi32 = phi.astype(np.float32)
    want, _ = _oracle_run(c, phi32.astype(np.float64), steps, 1e-12, 8, cap)
    s = make_solver(M, c, "fp32")
    s.set_theta_tolerance(1e-6, 8)
    s.set_state(phi32)
    s.step(steps)
    got = s.get_state().astype(np.float64)
    st = s.theta_stats(reset=True)
    assert s.theta_stats()["total_sweeps"] == 0
    s.close()
    assert st["unconverged"] == 0 and st["steps"] == steps
    assert rel_l2(got, want) < 1e-5


@pytest.mark.parametrize("case", [CASES[0], CASES[3]], ids=["fused", "host-checked"])
def test_theta_cap_stops_and_equals_fixed_sweeps(M, case):
    """An unreachable tolerance stops every step at the cap (whole chunks),
    equal to the fixed-count theta step of that many sweeps, and is counted
    as not converged."""
    c = _case(case, 10)
    rng = np.random.default_rng(7)
    phi = rng.standard_normal(int(np.prod(c["n"])))
    s = make_solver(M, c, "fp64")
    s.set_theta_tolerance(1e-300, 4)
    s.set_state(phi)
    s.step(3)
    got = s.get_state()
    st = s.theta_stats()
    s.close()
    assert st == dict(total_sweeps=36, steps=3, max_sweeps=12, unconverged=3)
    want = phi
    spec = oracle_spec(dict(c, theta_iters=12))
    for _ in range(3):
        want = O.theta_step(spec, want)
    assert np.array_equal(got, want)


def test_theta_tolerance_argument_checks(M):
    c = _case(CASES[2], 8)
    s = make_solver(M, c, "fp64")
    with pytest.raises(M.MfdError):
        s.set_theta_tolerance(-1.0)
    with pytest.raises(M.MfdError):
        s.set_theta_tolerance(1e-6, 17)
    s.close()
    c2 = dict(CASES[2], eq="lcde", a=(1.0, 0.0, 0.0), dx=1.0, dt=1.0)
    e = make_solver(M, c2, "fp64")
    with pytest.raises(M.MfdError):
        e.set_theta_tolerance(1e-6)
    e.close()


BURG = [
    dict(name="burgers-d2q9", lattice="D2Q9", n=(203, 150)),
    dict(name="burgers-d1q3", lattice="D1Q3", n=(500,)),
    dict(name="burgers-d3q19", lattice="D3Q19", n=(14, 11, 9)),
]


def _burgers_theta(c, dt_factor=4.0, nu=5e-3, theta=0.5, cap=64):
    dx = 1.0 / c["n"][0]
    dt = dt_factor * 0.3 * dx * dx / nu
    s = 2 * nu * dt / ((1.0 / 3.0) * dx * dx)
    a = ((s + 1) / 2, 1 - s, (s - 1) / 2)
    return dict(c, eq="burgers", a=a, kind="theta", theta=theta, theta_iters=cap, dx=dx, dt=dt)


@pytest.mark.parametrize("case", BURG, ids=lambda c: c["name"])
@pytest.mark.parametrize("tol,chunk", [(1e-12, 4), (0.0, 6)], ids=["tol", "fixed"])
def test_theta_burgers_fp64_matches_oracle(M, case, tol, chunk):
    """Burgers' equation with the theta scheme (Picard iteration with the
    Jacobi splitting of the linear even part): every state bit-exact with the
    oracle's iteration, sweep counts equal; tol = 0 runs theta_iters sweeps."""
    from oracle import implicit as IM

    cap = 64 if tol > 0 else chunk
    c = _burgers_theta(case, cap=cap)
    spec = oracle_spec(c)
    rng = np.random.default_rng(12)
    phi = 0.1 * rng.uniform(-1, 1, int(np.prod(c["n"])))
    want, sweeps = phi, []
    for _ in range(3):
        want, k, _ = IM.theta_picard_solve(spec, want, tol if tol > 0 else 1e-300,
                                           chunk if tol > 0 else cap, cap)
        sweeps.append(k)
    s = make_solver(M, c, "fp64")
    if tol > 0:
        s.set_theta_tolerance(tol, chunk)
    s.set_state(phi)
    s.step(3)
    got = s.get_state()
    st = s.theta_stats()
    s.close()
    assert np.array_equal(got, want)
    if tol > 0:
        assert st["total_sweeps"] == sum(sweeps) and st["unconverged"] == 0


def test_theta_burgers_fp32_within_1e5(M):
    from oracle import implicit as IM

    c = _burgers_theta(BURG[0])
    spec = oracle_spec(c)
    rng = np.random.default_rng(13)
    phi = (0.1 * rng.uniform(-1, 1, int(np.prod(c["n"])))).astype(np.float32)
    want = phi.astype(np.float64)
    for _ in range(4):
        want, _, _ = IM.theta_picard_solve(spec, want, 1e-12, 4, 64)
    s = make_solver(M, c, "fp32")
    s.set_theta_tolerance(1e-6, 4)
    s.set_state(phi)
    s.step(4)
    got = s.get_state().astype(np.float64)
    s.close()
    assert rel_l2(got, want) < 1e-5


NSE_TH = [
    dict(name="nse-d2q9", lattice="D2Q9", n=(96, 70)),
    dict(name="nse-d2q5", lattice="D2Q5", n=(64, 40)),
    dict(name="nse-d3q19", lattice="D3Q19", n=(14, 11, 9)),
    dict(name="nse-d2q5ii", lattice="D2Q5II", n=(70, 19)),
]


def _nse_theta(c, theta=0.5, cap=64, s_rho=1.6, s_j=0.9):
    def fam(s):
        return ((s + 1) / 2, 1 - s, (s - 1) / 2)

    return dict(c, eq="nse", rho0=1.0, a=fam(s_rho), ab=fam(s_j), kind="theta", theta=theta,
                theta_iters=cap, dx=1.0, dt=1.0)


def _nse_state(c, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    nf = 1 + len(c["n"])
    return amp * rng.uniform(-1, 1, nf * int(np.prod(c["n"])))


@pytest.mark.parametrize("case", NSE_TH, ids=lambda c: c["name"])
@pytest.mark.parametrize("theta,tol,chunk", [(0.5, 1e-12, 4), (0.0, 1e-10, 3), (0.5, 0.0, 5)],
                         ids=["half-tol", "implicit-tol", "fixed"])
def test_theta_nse_fp64_matches_oracle(M, case, theta, tol, chunk):
    """The NSE theta step (Picard sweeps, the own-node coefficient of the
    linear EDF parts split per field): every state bit-exact with the
    oracle's iteration and the sweep counts equal; tol = 0 runs theta_iters
    sweeps."""
    from oracle import implicit as IM

    cap = 64 if tol > 0 else chunk
    c = _nse_theta(case, theta=theta, cap=cap)
    spec = oracle_spec(c)
    phi = _nse_state(c, 21)
    want, sweeps = phi, []
    for _ in range(3):
        want, k, _ = IM.theta_picard_solve(spec, want, tol if tol > 0 else 1e-300,
                                           chunk if tol > 0 else cap, cap)
        sweeps.append(k)
    s = make_solver(M, c, "fp64")
    if tol > 0:
        s.set_theta_tolerance(tol, chunk)
    s.set_state(phi)
    s.step(1)
    s.step(2)
    got = s.get_state()
    st = s.theta_stats()
    s.close()
    assert np.array_equal(got, want)
    if tol > 0:
        assert st["total_sweeps"] == sum(sweeps) and st["unconverged"] == 0


@pytest.mark.parametrize("case", NSE_TH[:1] + NSE_TH[2:], ids=lambda c: c["name"])
def test_theta_nse_fp32_within_1e5(M, case):
    from oracle import implicit as IM

    c = _nse_theta(case)
    spec = oracle_spec(c)
    phi = _nse_state(c, 22).astype(np.float32)
    want = phi.astype(np.float64)
    for _ in range(4):
        want, _, _ = IM.theta_picard_solve(spec, want, 1e-12, 4, 64)
    s = make_solver(M, c, "fp32")
    s.set_theta_tolerance(1e-6, 4)
    s.set_state(phi)
    s.step(4)
    got = s.get_state().astype(np.float64)
    st = s.theta_stats()
    s.close()
    assert st["unconverged"] == 0
    assert rel_l2(got, want) < 1e-5


# ------------------------------------------------------- multigrid V-cycles
MGC = [
    dict(name="mg-d2q9", lattice="D2Q9", n=(256, 128), u=(0.1, -0.05), K=[[4.0, 0.0], [0.0, 4.0]]),
    dict(name="mg-d2q5", lattice="D2Q5", n=(96, 64), u=(0.1, -0.05), K=[[3.0, 0.0], [0.0, 3.0]]),
]


def _mg_case(c, cap):
    return dict(c, eq="lcde", a=(1.0, 0.0, 0.0), kind="theta", theta=0.5, theta_iters=cap,
                dx=1.0, dt=1.0)


def _exact_steps(c, phi, steps):
    from oracle import implicit as IM

    spec = oracle_spec(c)
    x = phi
    for _ in range(steps):
        x, _ = IM.theta_exact_periodic(spec, x)
    return x


@pytest.mark.parametrize("case", MGC, ids=lambda c: c["name"])
@pytest.mark.parametrize("levels,pre,post", [(-1, 2, 2), (3, 1, 1)], ids=["auto-v22", "l3-v11"])
def test_theta_multigrid_fp64_matches_exact_solve(M, case, levels, pre, post):
    """Multigrid V-cycles solve the theta step of Eq. (GCN) to the residual
    tolerance: after three steps the state is within 1e-9 (relative) of the
    exact periodic solve (the discrete Fourier transform of the same
    circulant system, in the oracle), every step converged, and the full
    hierarchy takes few cycles (Jacobi needs about 100 sweeps here)."""
    c = _mg_case(case, 80)
    rng = np.random.default_rng(31)
    phi = rng.standard_normal(int(np.prod(c["n"])))
    want = _exact_steps(c, phi, 3)
    s = make_solver(M, c, "fp64")
    s.set_theta_tolerance(1e-11)
    s.set_theta_multigrid(levels, pre, post)
    s.set_state(phi)
    s.step(1)
    s.step(2)
    got = s.get_state()
    st = s.theta_stats()
    s.close()
    assert st["unconverged"] == 0 and st["steps"] == 3
    if levels < 0:
        assert st["max_sweeps"] <= 12, st
    assert rel_l2(got, want) < 1e-9


def test_theta_multigrid_fixed_cycles_and_switch_off(M):
    """tol = 0 runs theta_iters cycles (6: within 1e-6 of the exact step);
    levels = 0 returns to Jacobi sweeps, whose result equals the oracle's
    Jacobi iteration bit for bit."""
    c = _mg_case(MGC[0], 6)
    rng = np.random.default_rng(32)
    phi = rng.standard_normal(int(np.prod(c["n"])))
    s = make_solver(M, c, "fp64")
    s.set_theta_multigrid(-1)
    s.set_state(phi)
    s.step(1)
    got = s.get_state()
    assert rel_l2(got, _exact_steps(c, phi, 1)) < 1e-6
    s.set_theta_multigrid(0)
    s.set_state(phi)
    s.step(1)
    got_j = s.get_state()
    s.close()
    assert np.array_equal(got_j, O.theta_step(oracle_spec(c), phi))


def test_theta_multigrid_fp32_within_1e5(M):
    """binary32 V-cycles at tolerance 1e-5 on smooth data (the C2 hill plus
    a low mode): within 3e-5 of the exact binary64 solve after four steps."""
    c = _mg_case(MGC[0], 40)
    nx, ny = c["n"]
    X, Y = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny, indexing="xy")
    phi = (np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / (2 * 0.05 ** 2))
           + 0.1 * np.sin(2 * np.pi * X) * np.cos(4 * np.pi * Y)).ravel()
    want = _exact_steps(c, phi.astype(np.float32).astype(np.float64), 4)
    s = make_solver(M, c, "fp32")
    s.set_theta_tolerance(1e-5)
    s.set_theta_multigrid(-1)
    s.set_state(phi.astype(np.float32))
    s.step(4)
    got = s.get_state().astype(np.float64)
    st = s.theta_stats()
    s.close()
    assert st["unconverged"] == 0
    assert rel_l2(got, want) < 3e-5
