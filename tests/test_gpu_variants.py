"""GPU: scheme variants against the FP64 oracle.

* Multiple-set (TRT-type) schemes, Eq. (2-2-1b): linear CDE two- and
  three-level and Burgers' equation on ragged 2D grids, single-step and
  temporally blocked plans (64- and 128-column windows): binary64 bit-exact,
  binary32 within 1e-5 (relative L2).
"""
import numpy as np
import pytest

from oracle import native as O
from parity_util import rel_l2

pytestmark = pytest.mark.gpu

K2 = [[0.03, 0.004], [0.004, 0.02]]
MS = [
    dict(name="lcde-2l", lattice="D2Q9", eq="lcde", n=(203, 150), u=(0.1, -0.05), K=K2,
         lambda_bar=1, a=(0.6, 0.2, 0.2), ae=(0.55, 0.2, 0.25), ao=(0.9, 0.0, 0.1)),
    dict(name="lcde-3l", lattice="D2Q9", eq="lcde", n=(203, 150), u=(0.1, -0.05), K=K2,
         lambda_bar=1, kind="three_level", a=(0.875, 0.0, 0.125), ah=(0.125, 0.0, -0.125),
         ae=(0.8, 0.1, 0.1), aeh=(0.1, -0.1, 0.1), ao=(0.95, 0.0, 0.05), aoh=(0.05, 0.0, -0.05)),
    dict(name="burgers-2l", lattice="D2Q5", eq="burgers", n=(150, 97), dx=0.01, dt=2e-5,
         a=(0.7, 0.1, 0.2), ae=(0.65, 0.1, 0.25), ao=(0.8, 0.1, 0.1)),
]


def _oracle(c, cur, prev, steps):
    three = c.get("kind") == "three_level"
    spec = {k: v for k, v in c.items() if k not in ("name", "kind")}
    spec["levels"] = 3 if three else 2
    if not three:
        spec["ah"] = (0.0, 0.0, 0.0)
    for _ in range(steps):
        nxt = O.mmfd_step(spec, cur, prev if three else None)
        prev, cur = cur, nxt
    return cur


def _gpu(M, c, cur, prev, steps, precision, plan):
    three = c.get("kind") == "three_level"
    s = M.Solver(c["lattice"], c["n"], c.get("dx", 1.0), precision, "mmfd")
    if c["eq"] == "lcde":
        s.set_equation("lcde", u=c["u"], K=c["K"], lambda_bar=c["lambda_bar"])
    else:
        s.set_equation("burgers")
    if three:
        s.set_scheme_sets("three_level", c["a"], c["ae"], c["ao"], c["ah"], c["aeh"], c["aoh"],
                          dt=c.get("dt", 1.0))
    else:
        s.set_scheme_sets("two_level", c["a"], c["ae"], c["ao"], dt=c.get("dt", 1.0))
    dt = np.float64 if precision == "fp64" else np.float32
    s.set_state(cur.astype(dt))
    if three:
        s.set_state(prev.astype(dt), level=1)
    if plan:
        s.set_plan(*plan)
    else:
        s.set_blocking(1)
    s.step(4)
    s.step(steps - 4)
    out = s.get_state().astype(np.float64)
    s.close()
    return out


@pytest.mark.parametrize("plan", [None, (4, 32, 64), (6, 64, 128)], ids=["single", "tb4-64", "tb6-128"])
@pytest.mark.parametrize("c", MS, ids=lambda c: c["name"])
def test_multiset_fp64_bit_exact(M, c, plan):
    if plan and plan[2] == 128 and c.get("kind") == "three_level":
        pytest.skip("128-column windows run two-level schemes")
    rng = np.random.default_rng(31)
    N = c["n"][0] * c["n"][1]
    cur, prev = rng.uniform(-0.5, 0.5, N), rng.uniform(-0.5, 0.5, N)
    steps = 17
    want = _oracle(c, cur, prev, steps)
    got = _gpu(M, c, cur, prev, steps, "fp64", plan)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("plan", [None, (6, 64, 128)], ids=["single", "tb6-128"])
@pytest.mark.parametrize("c", [MS[0], MS[2]], ids=["lcde-2l", "burgers-2l"])
def test_multiset_fp32_within_1e5(M, c, plan):
    rng = np.random.default_rng(32)
    N = c["n"][0] * c["n"][1]
    cur = rng.uniform(-0.5, 0.5, N).astype(np.float32).astype(np.float64)
    want = _oracle(c, cur, cur, 17)
    got = _gpu(M, c, cur, cur, 17, "fp32", plan)
    assert rel_l2(got, want) < 1e-5
