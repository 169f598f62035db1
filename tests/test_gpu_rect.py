"""GPU: rectangular lattices of Appendix A (spacing and d0 per axis) for the
linear CDE.  The kernels are the square lattice's; the per-axis values live
in the constant tables (bit-identical to the oracle's, tested on the CPU),
so binary64 runs equal the oracle's steps bit for bit under every launch
path: single steps, blocked plans (64- and 128-column windows), MesoFD,
three-level schemes, 3D grids and the theta step (Jacobi and multigrid)."""
import numpy as np
import pytest

from oracle import native as O
from parity_util import make_solver, oracle_spec, rand_state, rel_l2, run_oracle

pytestmark = pytest.mark.gpu

K2 = [[0.3, 0.05], [0.05, 0.2]]
CASES = [
    dict(name="d2q9-2l", lattice="D2Q9", n=(150, 97), u=(0.3, -0.2), K=K2, lambda_bar=1,
         dxv=(0.5, 2.0), d0v=(0.3, 0.45), dt=0.05, a=(1.0, 0.0, 0.0)),
    dict(name="d2q9-3l", lattice="D2Q9", n=(131, 70), u=(0.2, 0.1), K=K2, lambda_bar=1,
         dxv=(1.0, 0.75), d0v=(0.35, 0.3), dt=0.2, a=(0.875, 0.0, 0.125), ah=(0.125, 0.0, -0.125),
         kind="three_level"),
    dict(name="d2q5-2l", lattice="D2Q5", n=(129, 66), u=(0.3, -0.2), K=[[0.3, 0.0], [0.0, 0.2]],
         dxv=(1.0, 1.5), d0v=(0.3, 0.2), dt=0.2, a=(1.0, 0.0, 0.0)),
    dict(name="d2q9-mesofd", lattice="D2Q9", n=(100, 67), u=(0.3, -0.2), K=K2, lambda_bar=1,
         dxv=(0.5, 2.0), d0v=(0.3, 0.45), dt=0.05, a=(1.0, 0.0, 0.0), form="mesofd"),
    dict(name="d3q19", lattice="D3Q19", n=(21, 14, 11), u=(0.1, 0.2, -0.1),
         K=[[0.2, 0.01, 0.0], [0.01, 0.3, 0.02], [0.0, 0.02, 0.25]], lambda_bar=1,
         dxv=(1.0, 0.5, 2.0), d0v=(0.3, 0.25, 0.2), dt=0.05, a=(1.0, 0.0, 0.0)),
    dict(name="d3q7", lattice="D3Q7", n=(18, 13, 10), u=(0.1, 0.2, -0.1),
         K=[[0.15, 0.0, 0.0], [0.0, 0.25, 0.0], [0.0, 0.0, 0.1]], dxv=(1.0, 1.25, 0.75),
         d0v=(0.3, 0.2, 0.25), dt=0.1, a=(1.0, 0.0, 0.0)),
]


def _run(M, c, phi, steps, precision, plan=None):
    s = make_solver(M, c, precision)
    dt = np.float64 if precision == "fp64" else np.float32
    s.set_state(phi.astype(dt))
    if c.get("kind") == "three_level":
        s.set_state(phi.astype(dt), level=1)
    if plan is not None:
        s.set_plan(*plan)
    s.step(steps)
    out = s.get_state().astype(np.float64)
    s.close()
    return out


def _plans(c):
    if O.DIMS[c["lattice"]] != 2:
        return [None]
    if c.get("form") == "mesofd" or c.get("kind") == "three_level":
        return [None, (1, 0, 64), (4, 32, 64)]  # 128-column windows: two-level MMFD
    return [None, (1, 0, 64), (4, 32, 64), (6, 64, 128)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
def test_rect_fp64_bitwise(M, case):
    rng = np.random.default_rng(41)
    phi = rand_state(case, rng)
    steps = 9
    want = run_oracle(case, phi, phi, steps)
    for plan in _plans(case):
        got = _run(M, case, phi, steps, "fp64", plan)
        assert np.array_equal(got, want), plan


@pytest.mark.parametrize("case", CASES[:1] + CASES[4:5], ids=lambda c: c["name"])
def test_rect_fp32_within_1e5(M, case):
    rng = np.random.default_rng(42)
    phi = rand_state(case, rng)
    want = run_oracle(case, phi.astype(np.float32).astype(np.float64), None, 12)
    got = _run(M, case, phi, 12, "fp32")
    assert rel_l2(got, want) < 1e-5


def test_rect_theta_jacobi_and_multigrid(M):
    """theta = 0.5 on a rectangular D2Q9 grid: Jacobi sweeps equal the
    oracle's bit for bit; multigrid V-cycles reach the exact periodic solve
    (the Fourier solve of the same circulant system) within the tolerance."""
    from oracle import implicit as IM

    c = dict(CASES[0], n=(128, 64), d0v=(0.3, 0.05), kind="theta", theta=0.5, theta_iters=6,
             dt=0.5)
    rng = np.random.default_rng(43)
    phi = rng.standard_normal(128 * 64)
    spec = oracle_spec(c)
    want_j = O.theta_step(spec, phi)
    s = make_solver(M, c, "fp64")
    s.set_state(phi)
    s.step(1)
    assert np.array_equal(s.get_state(), want_j)
    s.close()
    c = dict(c, theta_iters=40)
    want, _ = IM.theta_exact_periodic(oracle_spec(c), phi)
    s = make_solver(M, c, "fp64")
    s.set_theta_tolerance(1e-11)
    s.set_theta_multigrid(-1)
    s.set_state(phi)
    s.step(1)
    got = s.get_state()
    st = s.theta_stats()
    s.close()
    assert st["unconverged"] == 0
    assert rel_l2(got, want) < 1e-9
