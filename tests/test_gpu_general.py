"""GPU: the general-scheme solver (mfd_general_*: stencil reach m, n time
levels, the linear CDE, every lattice of Appendix A with rD3Q27, square or
rectangular).  binary64 runs equal the oracle's central form
(oracle/general.py, pinned against the population-sum form and the
physical diffusion) bit for bit over several steps with the level ring
turning; binary32 stays within 1e-5; m = 1 with one or two levels matches
the regular solver's step."""
import numpy as np
import pytest

from oracle import general as GN
from oracle import native as O
from parity_util import make_solver, rel_l2

pytestmark = pytest.mark.gpu


def _a(rng, m, n):
    a = rng.uniform(-0.2, 0.5, (n, 2 * m + 1))
    a[0, m] += 1.0 - a.sum()  # A00 = 1
    A00, A10, A11, A22 = GN.moments(a)
    if not (A10 < 0 < A22):
        a[0, m - 1] += 1.0
        a[0, m] -= 1.0
    return a


CASES = [
    dict(name="d2q9-m2", lattice="D2Q9", n=(70, 45), m=2, nl=1),
    dict(name="d2q9-m3-n2", lattice="D2Q9", n=(66, 39), m=3, nl=2),
    dict(name="d2q5-m1-n3", lattice="D2Q5", n=(71, 40), m=1, nl=3),
    dict(name="d1q3-m3-n4", lattice="D1Q3", n=(301,), m=3, nl=4),
    dict(name="d3q19-m2", lattice="D3Q19", n=(20, 15, 12), m=2, nl=1),
    dict(name="d3q27-m1", lattice="D3Q27", n=(21, 14, 11), m=1, nl=1),
    dict(name="d3q27-m2-n2", lattice="D3Q27", n=(17, 13, 10), m=2, nl=2),
    dict(name="rect-d2q9-m2-n2", lattice="D2Q9", n=(64, 50), m=2, nl=2, spacing=(0.5, 2.0),
         d0v=(0.3, 0.45)),
    dict(name="rect-d3q27-m1-n2", lattice="D3Q27", n=(16, 12, 10), m=1, nl=2,
         spacing=(1.0, 0.5, 2.0), d0v=(0.3, 0.4, 0.5)),
    # extents below m + (nodes per thread): the wrap by remainder
    dict(name="tiny-d2q9-m3-n2", lattice="D2Q9", n=(5, 4), m=3, nl=2),
    dict(name="tiny-d2q9-m1", lattice="D2Q9", n=(70, 6), m=1, nl=1),
    dict(name="tiny-d3q27-m1", lattice="D3Q27", n=(6, 5, 3), m=1, nl=1),
    dict(name="tiny-d2q5-m2", lattice="D2Q5", n=(3, 2), m=2, nl=1),
]


def _spec(c):
    dim = O.DIMS[c["lattice"]]
    s = dict(lattice=c["lattice"], eq="lcde", n=c["n"], dx=1.0, dt=0.1,
             u=[0.1, -0.05, 0.03][:dim],
             K=(np.eye(dim) * 0.3 + 0.02 * (np.ones((dim, dim)) - np.eye(dim))).tolist(),
             lambda_bar=1)
    if "spacing" in c:
        s.update(dxv=c["spacing"], d0v=c["d0v"])
    return s


def _gpu(M, c, spec, a, levels, steps, precision):
    g = M.General(c["lattice"], c["n"], spec["dx"], a, spec["dt"], u=spec["u"], K=spec["K"],
                  lambda_bar=spec["lambda_bar"], precision=precision,
                  spacing=c.get("spacing"), d0v=c.get("d0v"))
    g.set_level(0, levels[0])
    for l in range(1, len(levels)):
        g.set_level(l, levels[l])
    g.step(2)
    g.step(steps - 2)
    out = [g.get_level(l).astype(np.float64) for l in range(len(levels))]
    g.close()
    return out


def _oracle(spec, a, levels, steps):
    lev = [np.asarray(v, dtype=np.float64) for v in levels]
    for _ in range(steps):
        new = GN.mmfd_step(spec, lev, a)
        lev = [new] + lev[:-1]
    return lev


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
def test_general_fp64_bitwise(M, case):
    rng = np.random.default_rng(51)
    spec = _spec(case)
    a = _a(rng, case["m"], case["nl"])
    N = int(np.prod(case["n"]))
    levels = [rng.standard_normal(N) for _ in range(case["nl"])]
    want = _oracle(spec, a, levels, 5)
    got = _gpu(M, case, spec, a, levels, 5, "fp64")
    for l in range(case["nl"]):
        assert np.array_equal(got[l], want[l]), l


@pytest.mark.parametrize("case", [CASES[0], CASES[6]], ids=lambda c: c["name"])
def test_general_fp32_within_1e5(M, case):
    rng = np.random.default_rng(52)
    spec = _spec(case)
    a = _a(rng, case["m"], case["nl"])
    N = int(np.prod(case["n"]))
    levels = [rng.standard_normal(N).astype(np.float32) for _ in range(case["nl"])]
    want = _oracle(spec, a, levels, 5)
    got = _gpu(M, case, spec, a, levels, 5, "fp32")
    assert rel_l2(got[0], want[0]) < 1e-5


@pytest.mark.parametrize("three", [False, True])
def test_general_m1_matches_the_regular_solver(M, three):
    """m = 1: the two-level (one row) and three-level (two rows) scheme of
    the regular solver, to rounding (the operations are grouped differently)."""
    c = dict(lattice="D2Q9", n=(96, 70), m=1, nl=2 if three else 1)
    spec = _spec(c)
    a = np.array([[0.875, 0.25, -0.125], [0.125, -0.25, 0.125]]) if three else np.array([[1.0, 0.0, 0.0]])
    rng = np.random.default_rng(53)
    phi = rng.standard_normal(96 * 70)
    got = _gpu(M, c, spec, a, [phi] * c["nl"], 6, "fp64")[0]
    case = dict(lattice="D2Q9", n=(96, 70), dx=1.0, dt=spec["dt"], u=spec["u"], K=spec["K"],
                lambda_bar=1, a=tuple(a[0]), kind="three_level" if three else "two_level")
    if three:
        case["ah"] = tuple(a[1])
    s = make_solver(M, case, "fp64")
    s.set_state(phi)
    s.step(6)
    want = s.get_state()
    s.close()
    assert np.allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


NLC = [
    dict(name="burgers-d2q9-m2", lattice="D2Q9", n=(66, 41), eq="burgers", m=2, nl=1),
    dict(name="burgers-d1q3-m3-n2", lattice="D1Q3", n=(257,), eq="burgers", m=3, nl=2),
    dict(name="nse-d2q9-m2-n2", lattice="D2Q9", n=(64, 45), eq="nse", m=2, nl=2),
    dict(name="nse-d3q19-m1-n3", lattice="D3Q19", n=(17, 12, 9), eq="nse", m=1, nl=3),
    dict(name="nse-d2q5-m3", lattice="D2Q5", n=(50, 37), eq="nse", m=3, nl=1),
    # extents below the reach: the tile's halo wraps more than once
    dict(name="tiny-nse-d2q9-m3-n2", lattice="D2Q9", n=(5, 3), eq="nse", m=3, nl=2),
    dict(name="tiny-burgers-d2q9-m2", lattice="D2Q9", n=(66, 2), eq="burgers", m=2, nl=1),
]


def _nl_case(c, rng):
    m, nl = c["m"], c["nl"]
    a = _a(rng, m, nl)
    ab = _a(rng, m, nl) if c["eq"] == "nse" else None
    spec = dict(lattice=c["lattice"], eq=c["eq"], n=c["n"], dx=1.0, dt=1.0, rho0=1.0, beta=1.0)
    N = int(np.prod(c["n"]))
    nf = 1 + len(c["n"]) if c["eq"] == "nse" else 1
    levels = [0.05 * rng.uniform(-1, 1, nf * N) for _ in range(nl)]
    return spec, a, ab, levels


def _nl_gpu(M, c, spec, a, ab, levels, steps, precision):
    g = M.General(c["lattice"], c["n"], 1.0, a, 1.0, eq=c["eq"], ab=ab, rho0=1.0,
                  precision=precision)
    g.set_level(0, levels[0])
    for l in range(1, len(levels)):
        g.set_level(l, levels[l])
    g.step(steps)
    out = [g.get_level(l).astype(np.float64) for l in range(len(levels))]
    g.close()
    return out


def _nl_oracle(spec, a, ab, levels, steps):
    lev = [np.asarray(v, dtype=np.float64) for v in levels]
    for _ in range(steps):
        lev = [GN.nonlinear_mmfd_step(spec, lev, a, ab)] + lev[:-1]
    return lev


@pytest.mark.parametrize("case", NLC, ids=lambda c: c["name"])
def test_general_nonlinear_fp64_bitwise(M, case):
    rng = np.random.default_rng(61)
    spec, a, ab, levels = _nl_case(case, rng)
    want = _nl_oracle(spec, a, ab, levels, 4)
    got = _nl_gpu(M, case, spec, a, ab, levels, 4, "fp64")
    for l in range(case["nl"]):
        assert np.array_equal(got[l], want[l]), l


@pytest.mark.parametrize("case", [NLC[0], NLC[2]], ids=lambda c: c["name"])
def test_general_nonlinear_fp32_within_1e5(M, case):
    rng = np.random.default_rng(62)
    spec, a, ab, levels = _nl_case(case, rng)
    levels = [v.astype(np.float32).astype(np.float64) for v in levels]
    want = _nl_oracle(spec, a, ab, levels, 4)
    got = _nl_gpu(M, case, spec, a, ab, levels, 4, "fp32")
    assert rel_l2(got[0], want[0]) < 1e-5


def test_general_nonlinear_refusals(M):
    """The nonlinear equations run on square lattices of up to 19 velocities."""
    a = [[0.5, 0.2, 0.3]]
    with pytest.raises(M.MfdError):
        M.General("D3Q27", (6, 6, 6), 1.0, a, 1.0, eq="nse", rho0=1.0)
    with pytest.raises(M.MfdError):
        M.General("D2Q9", (8, 8), 1.0, a, 1.0, eq="burgers", spacing=(1.0, 2.0), d0v=(0.3, 0.3))
