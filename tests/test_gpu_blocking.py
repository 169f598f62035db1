"""GPU: temporal blocking (MMFD and MesoFD), autotuning, reductions and the binary32 MesoFD
mass balance.

* Blocked LCDE and Burgers steps (depth 2, 4, 6, 8) equal the FP64 oracle
  value for value and equal the unblocked binary32 run bit for bit (one
  expression tree).
* Autotuning leaves the state untouched.
* FP64 reductions (mass, residual) agree with the oracle's compensated sums.
"""
import numpy as np
import pytest

from parity_util import rand_state, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

K2 = [[0.3, 0.04], [0.04, 0.2]]
BASE = dict(lattice="D2Q9", eq="lcde", u=(0.1, -0.07), K=K2, lambda_bar=1)
SCHEMES = {
    "2l": dict(a=(1.0, 0.0, 0.0)),
    "3l-trt": dict(kind="three_level", a=(1.0, 0.0, 0.4), ah=(0.0, -0.4, 0.0)),
    "3l-stencil": dict(kind="three_level", a=(0.875, 0.0, 0.125), ah=(0.125, 0.0, -0.125)),
}


def _burgers_a(n0, nu=5e-3):
    dx = 1.0 / n0
    dt = 0.5 * min(0.3 * dx * dx / nu, nu / 0.25)
    s = 2 * nu * dt / ((1.0 / 3.0) * dx * dx)
    return dict(dx=dx, dt=dt, a=((s + 1) / 2, 1 - s, (s - 1) / 2))


def _case(name, n):
    if name.startswith("burgers"):
        c = dict(lattice="D2Q9", eq="burgers", n=n, name=name, **_burgers_a(n[0]))
        if name == "burgers-3l":
            c.update(kind="three_level", a=(0.875, 0.0, 0.125), ah=(0.125, 0.0, -0.125))
        return c
    return dict(BASE, n=n, name=name, **SCHEMES[name])


ALL = list(SCHEMES) + ["burgers-2l", "burgers-3l"]


@pytest.mark.parametrize("tb", [2, 4, 6, 8])
@pytest.mark.parametrize("name", ALL)
@pytest.mark.parametrize("n", [(150, 77), (64, 32)])
def test_blocked_fp64_bitwise(M, tb, name, n):
    case = _case(name, n)
    print("case", name, tb, n, flush=True)
    rng = np.random.default_rng(5)
    cur, prev = rand_state(case, rng), rand_state(case, rng)
    steps = 3 * tb + 2
    want = run_oracle(case, cur, prev, steps)
    from parity_util import make_solver
    s = make_solver(M, case, "fp64")
    s.set_blocking(tb)
    s.set_state(cur)
    if case.get("kind") == "three_level":
        s.set_state(prev, level=1)
    s.step(steps)
    got = s.get_state()
    s.close()
    assert np.array_equal(got, want), np.abs(got - want).max()


@pytest.mark.parametrize("plan", [(4, 40, 128), (8, 48, 128), (2, 50, 128), (3, 32, 64)])
@pytest.mark.parametrize("name", ALL)
def test_explicit_plans_fp64_bitwise(M, plan, name):
    """Explicit launch plans, including 128-column windows, equal the oracle."""
    from parity_util import make_solver
    case = _case(name, (150, 77))
    print("case", name, plan, flush=True)
    rng = np.random.default_rng(15)
    cur, prev = rand_state(case, rng), rand_state(case, rng)
    steps = 2 * plan[0] + 3
    want = run_oracle(case, cur, prev, steps)
    s = make_solver(M, case, "fp64")
    s.set_plan(*plan)
    assert s.launch_plan() == plan
    s.set_state(cur)
    if case.get("kind") == "three_level":
        s.set_state(prev, level=1)
    s.step(steps)
    got = s.get_state()
    s.close()
    assert np.array_equal(got, want), np.abs(got - want).max()


NSE = {
    "nse-srt": dict(lattice="D2Q9", eq="nse", rho0=1.0, a=(1.0, 0.0, 0.0)),
    "nse-trt": dict(lattice="D2Q9", eq="nse", rho0=1.0, kind="three_level", a=(1.0, 0.0, 0.4),
                    ah=(0.0, -0.4, 0.0)),
    "nse-trt-heluo": dict(lattice="D2Q9", eq="nse", rho0=1.0, he_luo=1, kind="three_level",
                          a=(1.0, 0.0, 0.4), ah=(0.0, -0.4, 0.0)),
    "nse-d2q5-trt": dict(lattice="D2Q5", eq="nse", rho0=1.0, kind="three_level", a=(1.0, 0.0, 0.4),
                         ah=(0.0, -0.4, 0.0)),
}


@pytest.mark.parametrize("plan", [(2, 32, 64), (5, 32, 64), (12, 32, 64), (4, 64, 64), (28, 64, 64)])
@pytest.mark.parametrize("name", list(NSE))
@pytest.mark.parametrize("n", [(150, 77), (64, 64)])
def test_nse_blocked_fp64_bitwise(M, plan, name, n):
    """Blocked NSE launches (pair parts in LDS, moments in registers) equal
    the oracle value for value."""
    from parity_util import make_solver
    case = dict(NSE[name], n=n, name=name)
    print("case", name, plan, n, flush=True)
    rng = np.random.default_rng(17)
    cur, prev = rand_state(case, rng), rand_state(case, rng)
    pairs = 4 if case["lattice"] == "D2Q9" else 2
    if 2 * pairs * plan[1] * plan[2] * 8 > 160 * 1024:
        pytest.skip("window beyond the LDS in binary64")
    steps = 2 * plan[0] + 1
    want = run_oracle(case, cur, prev, steps)
    s = make_solver(M, case, "fp64")
    s.set_plan(*plan)
    s.set_state(cur)
    if case.get("kind") == "three_level":
        s.set_state(prev, level=1)
    s.step(steps)
    got = s.get_state()
    if case.get("kind") == "three_level":
        want_prev = run_oracle(case, cur, prev, steps - 1)
        assert np.array_equal(s.get_state(level=1), want_prev)
    s.close()
    assert np.array_equal(got, want), np.abs(got - want).max()


@pytest.mark.parametrize("name", list(NSE))
def test_nse_blocked_fp32_equals_unblocked(M, name):
    from parity_util import make_solver
    case = dict(NSE[name], n=(300, 140), name=name)
    rng = np.random.default_rng(18)
    cur = rand_state(case, rng).astype(np.float32)
    prev = rand_state(case, rng).astype(np.float32)
    outs = []
    for plan in ((1,), (4, 32, 64), (6, 64, 64)):
        s = make_solver(M, case, "fp32")
        s.set_plan(*plan)
        s.set_state(cur)
        if case.get("kind") == "three_level":
            s.set_state(prev, level=1)
        s.step(29)
        outs.append(s.get_state())
        s.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_plan_rejections(M):
    from parity_util import make_solver
    s = make_solver(M, _case("2l", (100, 77)), "fp32")
    for plan in ((4, 40, 128), (4, 80, 64), (4, 40, 96), (30, 80, 64), (4, 9, 64)):
        with pytest.raises(M.MfdError):
            s.set_plan(*plan)
    s.set_plan(1)
    assert s.launch_plan() == (1, 0, 0)
    s.close()


@pytest.mark.parametrize("name", ALL)
def test_blocked_fp32_equals_unblocked(M, name):
    from parity_util import make_solver
    case = _case(name, (300, 140))
    rng = np.random.default_rng(6)
    cur = rand_state(case, rng).astype(np.float32)
    prev = rand_state(case, rng).astype(np.float32)
    outs = []
    for tb in (1, 4, 8):
        s = make_solver(M, case, "fp32")
        s.set_blocking(tb)
        s.set_state(cur)
        if case.get("kind") == "three_level":
            s.set_state(prev, level=1)
        s.step(37)
        outs.append(s.get_state())
        s.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


MESO = {
    "lcde-d2q9": dict(BASE, a=(1.0, 0.0, 0.0)),
    "lcde-d2q9-a": dict(BASE, a=(0.9, 0.05, 0.1)),
    "lcde-d2q5": dict(BASE, lattice="D2Q5", K=[[0.3, 0.0], [0.0, 0.2]], a=(1.0, 0.0, 0.0)),
    "burgers-d2q9": dict(lattice="D2Q9", eq="burgers", **_burgers_a(150)),
    "burgers-beta-d2q9": dict(lattice="D2Q9", eq="burgers", beta=0.6, **_burgers_a(150)),
    "burgers-d2q5": dict(lattice="D2Q5", eq="burgers", **_burgers_a(150)),
}


def _meso_oracle(case, cur, steps):
    from oracle import native as O
    from parity_util import oracle_spec
    spec = oracle_spec(case)
    pop = O.init_populations(spec, cur)
    for _ in range(steps):
        pop, _ = O.mesofd_step(spec, pop, None)
    return pop, O.moments(spec, pop)


@pytest.mark.parametrize("plan", [(2, 32, 64), (3, 48, 64), (4, 40, 128), (8, 48, 128)])
@pytest.mark.parametrize("name", list(MESO))
@pytest.mark.parametrize("n", [(150, 77), (64, 32)])
def test_mesofd_blocked_fp64_bitwise(M, plan, name, n):
    """Blocked MesoFD launches (moments carried in the window, populations of
    the last step written out) equal the oracle: moments and populations,
    value for value, also after a ragged remainder of single steps."""
    from parity_util import make_solver
    if plan[1] > n[1] or plan[2] > n[0]:
        pytest.skip("window larger than the grid")
    case = dict(MESO[name], n=n, name=name, form="mesofd")
    print("case", name, plan, n, flush=True)
    rng = np.random.default_rng(19)
    cur = rand_state(case, rng)
    steps = 2 * plan[0] + 3
    pop, want = _meso_oracle(case, cur, steps)
    s = make_solver(M, case, "fp64")
    s.set_plan(*plan)
    assert s.launch_plan() == plan
    s.set_state(cur)
    s.step(steps)
    got = s.get_state()
    gpop = s.get_state(populations=True)
    s.close()
    assert np.array_equal(got, want), np.abs(got - want).max()
    assert np.array_equal(gpop, pop), np.abs(gpop - pop).max()


@pytest.mark.parametrize("name", list(MESO))
def test_mesofd_blocked_fp32_equals_unblocked(M, name):
    from parity_util import make_solver
    case = dict(MESO[name], n=(300, 140), name=name, form="mesofd")
    rng = np.random.default_rng(20)
    cur = rand_state(case, rng).astype(np.float32)
    outs = []
    for plan in ((1,), (4, 32, 64), (6, 64, 128), (12, 112, 128), (3, 10, 128), (16, 37, 128)):
        s = make_solver(M, case, "fp32")
        s.set_plan(*plan)
        s.set_state(cur)
        s.step(10)
        s.step(27)
        outs.append((s.get_state(), s.get_state(populations=True)))
        s.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0]) and np.array_equal(outs[0][1], o[1])


def test_mesofd_autotune_preserves_state(M):
    from parity_util import make_solver
    case = dict(MESO["lcde-d2q9"], n=(256, 128), form="mesofd")
    rng = np.random.default_rng(22)
    cur = rand_state(case, rng)
    s = make_solver(M, case, "fp64")
    s.set_state(cur)
    s.step(3)
    before = s.get_state(populations=True)
    s.autotune()
    assert np.array_equal(s.get_state(populations=True), before)
    s.step(11)
    pop, want = _meso_oracle(case, cur, 14)
    assert np.array_equal(s.get_state(), want)
    assert np.array_equal(s.get_state(populations=True), pop)
    s.close()


@pytest.mark.parametrize("plan", [(8, 128, 128), (10, 52, 128), (3, 10, 128), (16, 37, 128),
                                  (6, 99, 128), (12, 112, 128), (2, 20, 128)])
@pytest.mark.parametrize("lattice", ["D2Q9", "D2Q5"])
@pytest.mark.parametrize("eq", ["lcde", "burgers", "burgers-beta"])
def test_lane_shared_fp32_equals_unblocked(M, plan, lattice, eq):
    """The binary32 two-level windows whose lanes share neighbour values (128
    columns updated in place, two per lane: the linear CDE and Burgers with
    beta = 1; beta != 1 runs the general window) equal the single-step kernel
    bit for bit, on a grid with ragged tiles in both directions."""
    from parity_util import make_solver
    if eq == "lcde":
        K = K2 if lattice == "D2Q9" else [[0.3, 0.0], [0.0, 0.2]]
        case = dict(BASE, lattice=lattice, K=K, n=(301, 139), a=(1.0, 0.0, 0.0))
    else:
        case = dict(lattice=lattice, eq="burgers", n=(301, 139), **_burgers_a(301))
        if eq == "burgers-beta":
            case["beta"] = 0.6
    print("case", eq, lattice, plan, flush=True)
    rng = np.random.default_rng(23)
    cur = rand_state(case, rng).astype(np.float32)
    outs = []
    for p in ((1,), plan):
        s = make_solver(M, case, "fp32")
        s.set_plan(*p)
        assert s.launch_plan()[0] == p[0]
        s.set_state(cur)
        s.step(3 * plan[0] + 1)
        outs.append(s.get_state())
        s.close()
    assert np.array_equal(outs[0], outs[1]), np.abs(outs[0] - outs[1]).max()


@pytest.mark.parametrize("plan", [(8, 128, 128), (10, 52, 128), (3, 10, 128), (16, 37, 128),
                                  (12, 112, 128)])
@pytest.mark.parametrize("lattice", ["D2Q9", "D2Q5"])
@pytest.mark.parametrize("eq", ["lcde", "burgers", "burgers-beta"])
@pytest.mark.parametrize("form", ["mmfd", "mesofd"])
def test_lane_shared_fp64_bitwise(M, plan, lattice, eq, form):
    """The binary64 lane-shared windows (the node functions of the single-step
    kernels on values shared across lanes) equal the oracle value for value,
    moments and (MesoFD) populations, on a grid with ragged tiles in both
    directions and a ragged remainder of steps."""
    from parity_util import make_solver
    if eq == "lcde":
        K = K2 if lattice == "D2Q9" else [[0.3, 0.0], [0.0, 0.2]]
        case = dict(BASE, lattice=lattice, K=K, n=(301, 139), a=(1.0, 0.0, 0.0))
    else:
        case = dict(lattice=lattice, eq="burgers", n=(301, 139), **_burgers_a(301))
        if eq == "burgers-beta":
            case["beta"] = 0.6
    if form == "mesofd":
        case["form"] = "mesofd"
    print("case", form, eq, lattice, plan, flush=True)
    rng = np.random.default_rng(29)
    cur = rand_state(case, rng)
    steps = 2 * plan[0] + 3
    s = make_solver(M, case, "fp64")
    s.set_plan(*plan)
    assert s.launch_plan() == plan
    s.set_state(cur)
    s.step(steps)
    got = s.get_state()
    if form == "mesofd":
        pop, want = _meso_oracle(case, cur, steps)
        gpop = s.get_state(populations=True)
        s.close()
        assert np.array_equal(gpop, pop), np.abs(gpop - pop).max()
    else:
        want = run_oracle(case, cur, None, steps)
        s.close()
    assert np.array_equal(got, want), np.abs(got - want).max()


def _three_level_case(lattice, eq, hat):
    ah = {"trt": (0.0, -0.4, 0.0), "stencil": (0.125, 0.0, -0.125)}[hat]
    a = (1.0, 0.0, 0.4) if hat == "trt" else (0.875, 0.0, 0.125)
    if eq == "lcde":
        K = K2 if lattice == "D2Q9" else [[0.3, 0.0], [0.0, 0.2]]
        return dict(BASE, lattice=lattice, K=K, n=(301, 139), kind="three_level", a=a, ah=ah)
    case = dict(lattice=lattice, eq="burgers", n=(301, 139), **_burgers_a(301))
    case.update(kind="three_level", a=a, ah=ah)
    if eq == "burgers-beta":
        case["beta"] = 0.6
    return case


@pytest.mark.parametrize("plan", [(8, 48, 128), (10, 52, 128), (3, 10, 128), (16, 37, 128),
                                  (2, 20, 128)])
@pytest.mark.parametrize("lattice", ["D2Q9", "D2Q5"])
@pytest.mark.parametrize("eq", ["lcde", "burgers", "burgers-beta"])
@pytest.mark.parametrize("hat", ["trt", "stencil"])
def test_three_level_wide_fp64_bitwise(M, plan, lattice, eq, hat):
    """Three-level steps in 128-column windows (levels t, t - dt and the new
    one in LDS) equal the oracle value for value, both levels of the result,
    on a grid with ragged tiles in both directions and a ragged remainder of
    steps; the level t - dt enters through its centre value (trt) or through
    central differences (stencil)."""
    from parity_util import make_solver
    case = _three_level_case(lattice, eq, hat)
    print("case", hat, eq, lattice, plan, flush=True)
    rng = np.random.default_rng(31)
    cur, prev = rand_state(case, rng), rand_state(case, rng)
    steps = 2 * plan[0] + 3
    want = run_oracle(case, cur, prev, steps)
    want_prev = run_oracle(case, cur, prev, steps - 1)
    s = make_solver(M, case, "fp64")
    s.set_plan(*plan)
    assert s.launch_plan() == plan
    s.set_state(cur)
    s.set_state(prev, level=1)
    s.step(steps)
    got, got_prev = s.get_state(), s.get_state(level=1)
    s.close()
    assert np.array_equal(got, want), np.abs(got - want).max()
    assert np.array_equal(got_prev, want_prev), np.abs(got_prev - want_prev).max()


@pytest.mark.parametrize("plan", [(8, 104, 128), (12, 96, 128), (3, 10, 128), (16, 37, 128)])
@pytest.mark.parametrize("lattice", ["D2Q9", "D2Q5"])
@pytest.mark.parametrize("eq", ["lcde", "burgers-beta"])
@pytest.mark.parametrize("hat", ["trt", "stencil"])
def test_three_level_wide_fp32_equals_unblocked(M, plan, lattice, eq, hat):
    """The binary32 three-level windows equal the single-step kernel bit for
    bit (the same node function), both levels."""
    from parity_util import make_solver
    case = _three_level_case(lattice, eq, hat)
    print("case", hat, eq, lattice, plan, flush=True)
    rng = np.random.default_rng(37)
    cur = rand_state(case, rng).astype(np.float32)
    prev = rand_state(case, rng).astype(np.float32)
    outs = []
    for p in ((1,), plan):
        s = make_solver(M, case, "fp32")
        s.set_plan(*p)
        s.set_state(cur)
        s.set_state(prev, level=1)
        s.step(3 * plan[0] + 1)
        outs.append((s.get_state(), s.get_state(level=1)))
        s.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b), np.abs(a - b).max()


def test_three_level_window_limits(M):
    """Three levels of 128 columns in 160 KiB of LDS: up to 106 rows in
    binary32, 53 in binary64."""
    from parity_util import make_solver
    case = _three_level_case("D2Q9", "lcde", "stencil")
    s = make_solver(M, dict(case, n=(300, 200)), "fp32")
    s.set_plan(4, 106, 128)
    assert s.launch_plan() == (4, 106, 128)
    with pytest.raises(M.MfdError):
        s.set_plan(4, 108, 128)
    s.close()
    s = make_solver(M, dict(case, n=(300, 200)), "fp64")
    s.set_plan(4, 53, 128)
    assert s.launch_plan() == (4, 53, 128)
    with pytest.raises(M.MfdError):
        s.set_plan(4, 54, 128)
    s.close()


@pytest.mark.parametrize("plan", [(4, 40, 128), (3, 32, 64)])
@pytest.mark.parametrize("chunks", [(8,), (3, 8), (1, 1, 4)])
def test_mesofd_populations_of_the_last_step(M, plan, chunks):
    """Only the last step of each mfd_step call stores the populations (a
    blocked launch with steps after it in the call stores moments only): after
    calls that end in a blocked launch, in single steps, or in both, the
    populations read back equal the oracle's of the final step."""
    from parity_util import make_solver
    case = dict(MESO["lcde-d2q9"], n=(150, 77), name="lcde-d2q9", form="mesofd")
    rng = np.random.default_rng(47)
    cur = rand_state(case, rng)
    steps = sum(chunks)
    pop, want = _meso_oracle(case, cur, steps)
    s = make_solver(M, case, "fp64")
    s.set_plan(*plan)
    s.set_state(cur)
    for k in chunks:
        s.step(k)
    got, gpop = s.get_state(), s.get_state(populations=True)
    s.close()
    assert np.array_equal(got, want), np.abs(got - want).max()
    assert np.array_equal(gpop, pop), np.abs(gpop - pop).max()


def test_lane_shared_window_limits(M):
    """The in-place window holds at most 128 rows; other widths are rejected."""
    from parity_util import make_solver
    s = make_solver(M, dict(BASE, n=(300, 200), a=(1.0, 0.0, 0.0)), "fp32")
    for plan in ((4, 130, 128), (4, 40, 126), (4, 40, 96)):
        with pytest.raises(M.MfdError):
            s.set_plan(*plan)
    s.set_plan(4, 128, 128)
    assert s.launch_plan() == (4, 128, 128)
    s.close()


def test_autotune_preserves_state(M):
    from parity_util import make_solver
    case = _case("2l", (256, 128))
    rng = np.random.default_rng(7)
    cur = rand_state(case, rng)
    s = make_solver(M, case, "fp64")
    s.set_state(cur)
    s.step(5)
    before = s.get_state()
    d = s.autotune()
    assert d in (1, 2, 4, 6, 8, 10, 12, 14, 16)
    tb, h, w = s.launch_plan()
    assert tb == d and (h == 0) == (d == 1) and w in ((0,) if d == 1 else (64, 128))
    assert np.array_equal(s.get_state(), before)
    s.step(9)
    ref = make_solver(M, case, "fp64")
    ref.set_blocking(1)
    ref.set_state(cur)
    ref.step(14)
    assert np.array_equal(s.get_state(), ref.get_state())
    s.close()
    ref.close()


@pytest.mark.parametrize("form", ["mmfd", "mesofd"])
def test_reductions_match_oracle(M, form):
    from oracle import native as O
    from parity_util import make_solver
    case = dict(lattice="D2Q9", eq="nse", n=(70, 37), rho0=1.0, kind="three_level",
                a=(1.0, 0.0, 0.4), ah=(0.0, -0.4, 0.0), form=form)
    rng = np.random.default_rng(8)
    cur = rand_state(case, rng)
    s = make_solver(M, case, "fp64")
    s.set_state(cur)
    sums0, res0 = s.reduce()
    assert res0 == 0.0
    s.step(5)
    sums, res = s.reduce()
    want = run_oracle(case, cur, cur, 5)
    prev = run_oracle(case, cur, cur, 4)
    N = 70 * 37
    for f in range(3):
        w = O.csum(want[f * N:(f + 1) * N])
        assert abs(sums[f] - w) <= 1e-12 * (1 + np.abs(want[f * N:(f + 1) * N]).sum())
        # mass / momentum conserved over the run (prev == cur start)
        assert abs(sums[f] - sums0[f]) <= 1e-12 * (1 + np.abs(cur[f * N:(f + 1) * N]).sum())
    wres = float(np.linalg.norm(want[:N] - prev[:N]))
    assert abs(res - wres) <= 1e-12 * wres
    s.close()


def test_fp32_mesofd_mass_balance(M):
    """binary32 MesoFD keeps the zeroth moment: the rest population closes
    the EDF sum, so the mass drift is round-off noise, not a per-step bias."""
    from parity_util import make_solver
    n = 256
    case = dict(lattice="D2Q9", eq="lcde", n=(n, n), u=(0.05, 0.03), K=[[0.02, 0.005], [0.005, 0.01]],
                dx=1.0 / n, dt=16.0 / n ** 2, lambda_bar=1, a=(1.0, 0.0, 0.0), form="mesofd")
    rng = np.random.default_rng(9)
    phi = 1.0 + 0.1 * rng.standard_normal(n * n)
    s = make_solver(M, case, "fp32")
    s.set_state(phi.astype(np.float32))
    m0 = s.reduce()[0][0]
    s.step(2000)
    m1 = s.reduce()[0][0]
    s.close()
    assert abs(m1 - m0) / abs(m0) < 2e-5
