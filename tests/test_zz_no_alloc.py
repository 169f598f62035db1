"""GPU: mfd_step_noalloc (caller-owned levels, work levels in the library's
fixed device scratch) against mfd_set_state / mfd_step / mfd_get_state.

Two calls in a row share the scratch, the second on a smaller grid; each
result must equal the ordinary entry point's bit for bit (both precisions,
two- and three-level, blocked and single-step plans), and neither call may
change the device bytes the library or torch hold.
"""
import numpy as np
import pytest
import torch

from parity_util import make_solver, rand_state

pytestmark = pytest.mark.gpu

K2 = [[0.3, 0.04], [0.04, 0.2]]
TRT = ((1.0, 0.0, 0.4), (0.0, -0.4, 0.0))
EX13 = ((0.875, 0.0, 0.125), (0.125, 0.0, -0.125))

CASES = [
    # (first call, second call on a smaller grid)
    (dict(name="lcde-2l", lattice="D2Q9", n=(700, 515), eq="lcde", u=(0.1, -0.07), K=K2,
          lambda_bar=1, a=(1.0, 0.0, 0.0), steps=23),
     dict(name="lcde-2l-small", lattice="D2Q9", n=(130, 77), eq="lcde", u=(0.1, -0.07), K=K2,
          lambda_bar=1, a=(1.0, 0.0, 0.0), steps=9)),
    (dict(name="nse-3l", lattice="D2Q9", n=(300, 211), eq="nse", rho0=1.0, kind="three_level",
          a=TRT[0], ah=TRT[1], steps=11),
     dict(name="lcde-3l", lattice="D2Q9", n=(150, 77), eq="lcde", u=(0.1, -0.07), K=K2,
          lambda_bar=1, kind="three_level", a=EX13[0], ah=EX13[1], steps=13)),
    (dict(name="burgers-1d", lattice="D1Q3", n=(5000,), eq="burgers", dx=0.01, dt=1e-5,
          a=(0.55, -0.1, 0.55), steps=17),
     dict(name="nse-d3q19", lattice="D3Q19", n=(20, 13, 9), eq="nse", rho0=1.0, kind="three_level",
          a=TRT[0], ah=TRT[1], steps=5)),
]


def _ordinary(M, c, cur, prev, precision):
    s = make_solver(M, c, precision)
    dt = np.float64 if precision == "fp64" else np.float32
    s.set_state(cur.astype(dt))
    if c.get("kind") == "three_level":
        s.set_state(prev.astype(dt), level=1)
    s.step(c["steps"])
    out = (s.get_state(), s.get_state(level=1) if c.get("kind") == "three_level" else None)
    s.close()
    return out


def _noalloc(M, c, cur, prev, precision):
    s = make_solver(M, c, precision)
    tdt = torch.float64 if precision == "fp64" else torch.float32
    l0 = torch.tensor(cur, dtype=tdt, device="cuda")
    three = c.get("kind") == "three_level"
    l1 = torch.tensor(prev, dtype=tdt, device="cuda") if three else None
    torch.cuda.synchronize()
    lib0, _ = M.memory_stats()
    t0 = torch.cuda.memory_allocated()
    s.step_noalloc(l0.data_ptr(), l1.data_ptr() if three else None, c["steps"])
    s.synchronize()
    lib1, _ = M.memory_stats()
    t1 = torch.cuda.memory_allocated()
    out = (l0.cpu().numpy(), l1.cpu().numpy() if three else None)
    s.close()
    return out, (lib1 - lib0, t1 - t0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("pair", CASES, ids=lambda p: p[0]["name"])
def test_noalloc_equals_step(M, pair, precision):
    rng = np.random.default_rng(21)
    for c in pair:  # two calls in a row, the second smaller
        cur, prev = rand_state(c, rng), rand_state(c, rng)
        want = _ordinary(M, c, cur, prev, precision)
        got, (dlib, dtorch) = _noalloc(M, c, cur, prev, precision)
        assert dlib == 0 and dtorch == 0, c["name"]
        assert np.array_equal(got[0], want[0]), c["name"]
        if want[1] is not None:
            assert np.array_equal(got[1], want[1]), c["name"]


def test_noalloc_blocked_plan_and_limits(M):
    """A forced blocked plan (several launches plus a remainder) on the
    caller's levels; a state beyond the scratch limit and a missing level
    pointer are refused without touching the device."""
    c = dict(CASES[1][1], steps=15)
    rng = np.random.default_rng(22)
    cur, prev = rand_state(c, rng), rand_state(c, rng)
    s = make_solver(M, c, "fp64")
    s.set_plan(6, 48, 64)
    s.set_state(cur)
    s.set_state(prev, level=1)
    s.step(15)
    want = s.get_state()
    l0 = torch.tensor(cur, dtype=torch.float64, device="cuda")
    l1 = torch.tensor(prev, dtype=torch.float64, device="cuda")
    s.step_noalloc(l0.data_ptr(), l1.data_ptr(), 15)
    s.synchronize()
    assert np.array_equal(l0.cpu().numpy(), want)
    assert np.array_equal(s.get_state(), want)  # the solver's own state is untouched
    with pytest.raises(M.MfdError) as ei:
        s.step_noalloc(l0.data_ptr(), None, 1)
    assert ei.value.code == M.MFD_E_ARG
    s.close()
    big = dict(CASES[0][0], n=(4096, 2049))
    b = make_solver(M, big, "fp32")
    x = torch.zeros(4096 * 2049, dtype=torch.float32, device="cuda")
    with pytest.raises(M.MfdError) as ei:
        b.step_noalloc(x.data_ptr(), None, 1)
    assert ei.value.code == M.MFD_E_ARG
    b.close()
