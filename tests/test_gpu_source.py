"""GPU: the source term of the linear CDE step (the b terms of Eq. (2-1) /
(3layerMMFD-1), F_j of Eq. (SourceF) with M_1F = v S, S = exp(lambda t) G).

* binary64 equals the oracle value for value on every lattice, for the
  two-level and three-level schemes of Example 1 and random coefficients, on
  ragged grids, with the steps split over several calls (the time of a step
  counts from the last set_state);
* binary32 stays within 1e-5 (relative L2) of the binary64 oracle;
* the MesoFD form (1D / 2D): moments and populations equal the oracle value
  for value;
* blocked source steps (several steps per launch, G staged once) equal the
  oracle value for value under every plan, split over calls;
* a launch plan the source step cannot take (128-column windows) is not
  used while the source is set;
* 3D MesoFD, other equations, the theta scheme and batches refuse it.
"""
import math

import numpy as np
import pytest

from oracle import native as O
from parity_util import make_solver, oracle_spec, rand_state, rel_l2

pytestmark = pytest.mark.gpu

K2 = [[0.02, 0.005], [0.005, 0.01]]
SCHEMES = {
    "srt": dict(a=(1.0, 0.0, 0.0)),
    "ex1-case2": dict(kind="three_level", a=(7 / 8, 1 / 4, -1 / 8), ah=(1 / 8, -1 / 4, 1 / 8)),
    "ex1-case3": dict(kind="three_level", a=(7 / 8, 0.0, 1 / 8), ah=(1 / 8, 0.0, -1 / 8)),
}
GRIDS = {
    "D1Q3": dict(n=(301,), u=(0.3,), K=[[0.02]], lambda_bar=1),
    "D2Q5": dict(n=(150, 77), u=(0.3, -0.2), K=[[0.02, 0.0], [0.0, 0.02]], lambda_bar=0),
    "D2Q9": dict(n=(150, 77), u=(0.3, -0.2), K=K2, lambda_bar=1),
    "D3Q19": dict(n=(20, 12, 9), u=(0.3, -0.2, 0.1), K=[[0.02, 0.0, 0.0], [0.0, 0.02, 0.0], [0.0, 0.0, 0.02]],
                  lambda_bar=1),
}
COEFS = {
    "example1": dict(b=(1.5, 0.0, 0.0), bh=(-0.5, 0.0, 0.0)),
    "random": dict(b=(0.3, 0.5, 0.2), bh=(0.1, -0.2, 0.05)),
}


def _case(lat, scheme):
    return dict(lattice=lat, eq="lcde", dx=0.05, dt=0.01, **GRIDS[lat], **SCHEMES[scheme])


def _oracle(case, cur, prev, steps, G, lam, coef, v):
    spec = oracle_spec(case)
    three = spec["levels"] == 3
    dt = case["dt"]
    for s in range(steps):
        src = dict(coef, v=v, S_t=math.exp(lam * (s * dt)) * G,
                   S_m=math.exp(lam * ((s - 1) * dt)) * G)
        nxt = O.mmfd_step(spec, cur, prev if three else None, src)
        prev, cur = cur, nxt
    return cur


def _gpu(M, case, cur, prev, chunks, G, lam, coef, v, precision="fp64", plan=None):
    s = make_solver(M, case, precision)
    dt = np.float64 if precision == "fp64" else np.float32
    if plan:
        s.set_plan(*plan)
    s.set_state(cur.astype(dt))
    if case.get("kind") == "three_level":
        s.set_state(prev.astype(dt), level=1)
    s.set_source(G, lam, coef["b"], coef["bh"], v)
    plan_seen = s.launch_plan()
    for k in chunks:
        s.step(k)
    out = s.get_state().astype(np.float64)
    s.close()
    return out, plan_seen


@pytest.mark.parametrize("lat", list(GRIDS))
@pytest.mark.parametrize("scheme", list(SCHEMES))
@pytest.mark.parametrize("coef", list(COEFS))
def test_source_fp64_bitwise(M, lat, scheme, coef):
    case = _case(lat, scheme)
    print("case", lat, scheme, coef, flush=True)
    rng = np.random.default_rng(41)
    cur, prev = rand_state(case, rng), rand_state(case, rng)
    G = rng.standard_normal(cur.size)
    v = tuple(rng.uniform(-0.5, 0.5, len(case["n"])))
    want = _oracle(case, cur, prev, 7, G, -0.7, COEFS[coef], v)
    got, _ = _gpu(M, case, cur, prev, (3, 4), G, -0.7, COEFS[coef], v)
    assert np.array_equal(got, want), np.abs(got - want).max()


def _oracle_meso(case, cur, prev, steps, G, lam, coef, v):
    spec = oracle_spec(case)
    three = spec["levels"] == 3
    dt = case["dt"]
    pop = O.init_populations(spec, cur)
    pm = prev if three else None
    for s in range(steps):
        src = dict(coef, v=v, S_t=math.exp(lam * (s * dt)) * G,
                   S_m=math.exp(lam * ((s - 1) * dt)) * G)
        pop, pm = O.mesofd_step(spec, pop, pm, src)
    return pop, O.moments(spec, pop)


@pytest.mark.parametrize("lat", ["D1Q3", "D2Q5", "D2Q9"])
@pytest.mark.parametrize("scheme", list(SCHEMES))
@pytest.mark.parametrize("coef", list(COEFS))
def test_source_mesofd_fp64_bitwise(M, lat, scheme, coef):
    """MesoFD with the source: moments and populations equal the oracle value
    for value, with the steps split over calls."""
    case = dict(_case(lat, scheme), form="mesofd")
    print("case mesofd", lat, scheme, coef, flush=True)
    rng = np.random.default_rng(45)
    cur, prev = rand_state(case, rng), rand_state(case, rng)
    G = rng.standard_normal(cur.size)
    v = tuple(rng.uniform(-0.5, 0.5, len(case["n"])))
    pop, want = _oracle_meso(case, cur, prev, 7, G, -0.7, COEFS[coef], v)
    s = make_solver(M, case, "fp64")
    s.set_state(cur)
    if case.get("kind") == "three_level":
        s.set_state(prev, level=1)
    s.set_source(G, -0.7, COEFS[coef]["b"], COEFS[coef]["bh"], v)
    s.step(3)
    s.step(4)
    got, gpop = s.get_state(), s.get_state(populations=True)
    s.close()
    assert np.array_equal(got, want), np.abs(got - want).max()
    assert np.array_equal(gpop, pop), np.abs(gpop - pop).max()


@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_source_fp32_tolerance(M, scheme):
    case = _case("D2Q9", scheme)
    rng = np.random.default_rng(42)
    cur, prev = rand_state(case, rng), rand_state(case, rng)
    G = rng.standard_normal(cur.size)
    want = _oracle(case, cur, prev, 40, G, 0.4, COEFS["example1"], (0.2, 0.1))
    got, _ = _gpu(M, case, cur, prev, (40,), G, 0.4, COEFS["example1"], (0.2, 0.1), "fp32")
    err = rel_l2(got, want)
    print("fp32 rel L2", scheme, err)
    assert err < 1e-5


def test_source_overrides_plan(M):
    """A 128-column plan set before the source is not used while the source
    is set (the source step takes 64-column windows of the same depth), and
    comes back when the source is cleared."""
    case = _case("D2Q9", "srt")
    rng = np.random.default_rng(43)
    cur = rand_state(case, rng)
    G = rng.standard_normal(cur.size)
    want = _oracle(case, cur, cur, 9, G, -0.2, COEFS["example1"], (0.1, 0.3))
    got, plan = _gpu(M, case, cur, cur, (9,), G, -0.2, COEFS["example1"], (0.1, 0.3),
                     plan=(4, 40, 128))
    assert plan[0] == 4 and plan[2] == 64
    assert np.array_equal(got, want)
    s = make_solver(M, case, "fp64")
    s.set_plan(4, 40, 128)
    s.set_state(cur)
    s.set_source(G)
    assert s.launch_plan()[2] == 64
    with pytest.raises(M.MfdError):
        s.set_plan(4, 40, 128)
    s.clear_source()
    assert s.launch_plan() == (4, 40, 128)
    s.close()


SRC_PLANS = [(1,), (2, 32), (4, 48), (6, 64), (8, 72), (16, 40)]


@pytest.mark.parametrize("plan", SRC_PLANS, ids=lambda p: "tb%d" % p[0])
@pytest.mark.parametrize("lat,scheme", [("D2Q9", "srt"), ("D2Q9", "ex1-case2"), ("D2Q5", "ex1-case3"),
                                        ("D2Q9", "ex1-case3")])
def test_source_blocked_fp64_bitwise(M, lat, scheme, plan):
    """The blocked source step (G staged once per launch, each step's factors
    exp(lambda t) from its own level's time): binary64 equal to the oracle
    for every plan, with blocks and a remainder split over calls."""
    case = _case(lat, scheme)
    print("case blocked source", lat, scheme, plan, flush=True)
    rng = np.random.default_rng(46)
    cur, prev = rand_state(case, rng), rand_state(case, rng)
    G = rng.standard_normal(cur.size)
    v = tuple(rng.uniform(-0.5, 0.5, 2))
    want = _oracle(case, cur, prev, 37, G, 0.7, COEFS["random"], v)
    got, seen = _gpu(M, case, cur, prev, (5, 32), G, 0.7, COEFS["random"], v,
                     plan=plan if len(plan) == 1 else (plan[0], plan[1], 64))
    assert seen[0] == plan[0]
    assert np.array_equal(got, want), np.abs(got - want).max()


@pytest.mark.parametrize("scheme", ["srt", "ex1-case2"])
def test_source_blocked_fp32_tolerance(M, scheme):
    case = _case("D2Q9", scheme)
    rng = np.random.default_rng(47)
    cur, prev = rand_state(case, rng), rand_state(case, rng)
    G = rng.standard_normal(cur.size)
    want = _oracle(case, cur, prev, 40, G, 0.4, COEFS["example1"], (0.2, 0.1))
    got, seen = _gpu(M, case, cur, prev, (40,), G, 0.4, COEFS["example1"], (0.2, 0.1), "fp32",
                     plan=(6, 64, 64))
    assert seen[0] == 6
    assert rel_l2(got, want) < 1e-5


def test_source_rejections(M):
    rng = np.random.default_rng(44)
    base = _case("D2Q9", "srt")
    G = rng.standard_normal(int(np.prod(base["n"])))
    G3 = rng.standard_normal(int(np.prod(GRIDS["D3Q19"]["n"])))
    for case, g in ((dict(_case("D3Q19", "srt"), form="mesofd"), G3),
                    (dict(lattice="D2Q9", eq="burgers", n=base["n"], dx=0.05, dt=0.001,
                          a=(1.0, 0.0, 0.0)), G),
                    (dict(base, kind="theta", theta=0.5, theta_iters=2), G)):
        s = make_solver(M, case, "fp64")
        with pytest.raises(M.MfdError):
            s.set_source(g)
        s.close()
    s = make_solver(M, base, "fp64")
    with pytest.raises(M.MfdError):
        s.set_source(G[:-1])
    bad = G.copy()
    bad[5] = np.nan
    with pytest.raises(M.MfdError):
        s.set_source(bad)
    s.set_state(rand_state(base, rng))
    s.set_source(G)
    b = M.Batch()
    with pytest.raises(M.MfdError):
        b.add(s, 10)
    b.close()
    s.close()
