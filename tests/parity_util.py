"""Shared helpers of the parity tests: one plain case description drives both
the FP64 oracle and the HIP library (each derives its own constants)."""
from __future__ import annotations

import numpy as np

from oracle import native as O


def rand_state(case, rng, scale=1.0):
    N = int(np.prod(case["n"]))
    dim = O.DIMS[case["lattice"]]
    eq = case.get("eq", "lcde")
    if eq == "lcde":
        return rng.standard_normal(N) * scale
    if eq == "burgers":
        return rng.uniform(-0.5, 0.5, N) * scale
    base = 1.0 if case.get("rho0", 0.0) == 0.0 else 0.0
    return np.concatenate([base + rng.uniform(-0.02, 0.02, N), rng.uniform(-0.05, 0.05, dim * N)])


def oracle_spec(case):
    keys = ("lattice", "n", "d0", "dx", "dt", "eq", "a", "ah", "ab", "abh", "u", "K", "lambda_bar",
            "beta", "rho0", "he_luo", "theta", "theta_iters", "d0v", "dxv")
    spec = {k: case[k] for k in keys if k in case}
    spec["levels"] = 3 if case.get("kind") == "three_level" else 2
    if case.get("kind") != "three_level":
        spec["ah"] = (0.0, 0.0, 0.0)
        spec.pop("abh", None)
    return spec


def run_oracle(case, cur, prev, steps):
    spec = oracle_spec(case)
    form = case.get("form", "mmfd")
    three = spec["levels"] == 3
    if case.get("kind") == "theta":
        for _ in range(steps):
            cur = O.theta_step(spec, cur)
        return cur
    if form == "mmfd":
        for _ in range(steps):
            nxt = O.mmfd_step(spec, cur, prev if three else None)
            prev, cur = cur, nxt
        return cur
    pop = O.init_populations(spec, cur)
    pm = prev if three else None
    for _ in range(steps):
        pop, pm = O.mesofd_step(spec, pop, pm)
    return O.moments(spec, pop)


def make_solver(M, case, precision):
    s = M.Solver(case["lattice"], case["n"], case.get("dx", 1.0), precision, case.get("form", "mmfd"),
                 d0=case.get("d0", 1.0 / 3.0))
    if "dxv" in case or "d0v" in case:
        s.set_rectangular(case.get("dxv", [case.get("dx", 1.0)] * 3),
                          case.get("d0v", [case.get("d0", 1.0 / 3.0)] * 3))
    s.set_equation(case.get("eq", "lcde"), u=case.get("u", ()), K=case.get("K"),
                   lambda_bar=case.get("lambda_bar", 0), beta=case.get("beta", 1.0),
                   rho0=case.get("rho0", 0.0), he_luo=case.get("he_luo", 0))
    kind = case.get("kind", "two_level")
    s.set_scheme(kind, case["a"], case.get("ah") if kind == "three_level" else None,
                 case.get("ab"), case.get("abh") if kind == "three_level" else None,
                 theta=case.get("theta", 1.0), theta_iters=case.get("theta_iters", 0),
                 dt=case.get("dt", 1.0))
    return s


def run_gpu(M, case, cur, prev, steps, precision="fp64", chunks=None):
    s = make_solver(M, case, precision)
    dt = np.float64 if precision == "fp64" else np.float32
    s.set_state(cur.astype(dt))
    if case.get("kind") == "three_level":
        s.set_state(prev.astype(dt), level=1)
    for k in (chunks or [steps]):
        s.step(k)
    out = s.get_state().astype(np.float64)
    s.close()
    return out


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
