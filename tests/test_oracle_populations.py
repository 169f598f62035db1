"""Pins of the oracle's per-direction MesoFD populations and of its
compensated sum.

* SRT with tau = 1 (a_{-1} = 1, every other coefficient 0) turns the MesoFD
  step of Eq. (2-1) into streaming of equilibria: f_j(x, t + dt) =
  f_j^eq(x - e_j, t) (the schemes written out for Case 1 of Examples 1 and
  2).  The oracle must reproduce it direction by direction, exactly.
* Exact rational brute force of every population of Eq. (2-1) /
  (3layer-1), with and without the b terms of the source (F_j of
  Eq. (SourceF)), on tiny periodic grids: the oracle's populations must lie
  within a few ulp of the rational values, direction by direction (a swapped
  direction or slot leaves the moments unchanged but fails here).
* The Neumaier-compensated sum against the exact (Fraction) sum of
  cancelling inputs, within the compensated-summation error bound.
"""
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import native as O
from tests.test_oracle_nonlinear import exact_edf, rand_state, to_fields
from tests.test_oracle_nonlinear import exact_weights as _weights_d1d2d3

EPS = np.finfo(float).eps


def exact_weights(lat):
    """Appendix A weights at d0 = 1/3 in exact arithmetic (rD2Q5I:
    w_0 = 1 - 2 d0, w_j = d0 / 2)."""
    if lat == "D2Q5":
        d = F(1, 3)
        return [1 - 2 * d] + [d / 2] * 4
    return _weights_d1d2d3(lat)


def _grid_shape(spec):
    n = list(spec["n"]) + [1] * (3 - len(spec["n"]))
    return n[2], n[1], n[0]


STREAM_CASES = [
    dict(lattice="D1Q3", eq="lcde", n=(7,), u=(0.1,), K=[[0.02]], dx=0.1, dt=0.05),
    dict(lattice="D2Q5", eq="lcde", n=(6, 5), u=(0.05, -0.02), K=[[0.01, 0.0], [0.0, 0.01]],
         dx=0.1, dt=0.05),
    dict(lattice="D2Q9", eq="lcde", n=(6, 5), u=(0.05, 0.03), K=[[0.02, 0.005], [0.005, 0.01]],
         lambda_bar=1, dx=0.05, dt=0.01),
    dict(lattice="D2Q9", eq="burgers", n=(5, 4), dx=0.5, dt=0.125),
    dict(lattice="D2Q9", eq="nse", n=(5, 4), rho0=1.0),
    dict(lattice="D3Q19", eq="nse", n=(4, 3, 3), rho0=1.0),
]


@pytest.mark.parametrize("spec", STREAM_CASES, ids=lambda s: "%s-%s" % (s["lattice"], s["eq"]))
def test_srt_tau1_streams_equilibria(spec):
    spec = dict(spec, a=(1.0, 0.0, 0.0))
    rng = np.random.default_rng(11)
    if spec["eq"] == "lcde":
        mom = rng.uniform(-1.0, 1.0, O.npoints(spec))
    else:
        mom = rand_state(spec, rng)
    pop = O.init_populations(spec, mom)
    new, _ = O.mesofd_step(spec, pop)
    # the step reads the EDF of the moments of `pop`
    feq = O.init_populations(spec, O.moments(spec, pop))
    E, _, _ = O.lattice_info(spec["lattice"])
    b = len(E)
    shape = _grid_shape(spec)
    N = O.npoints(spec)
    for j in range(b):
        g = feq[j * N:(j + 1) * N].reshape(shape)
        want = np.roll(g, shift=(int(E[j][2]), int(E[j][1]), int(E[j][0])), axis=(0, 1, 2))
        got = new[j * N:(j + 1) * N].reshape(shape)
        assert np.array_equal(got, want), "direction %d" % j


def exact_populations(spec, cur, prev, src=None):
    """Every population of Eq. (2-1) / (3layer-1) in rationals: list of b
    lists of N values.  `src` (linear CDE): dict(b, bh, v, S_t, S_m) adds
    dt sum_k [b_k F_j(x + k e_j, t) + bh_k F_j(x + k e_j, t - dt)] with
    F_j = w_j (S + e_j.(v dt/dx) S / d0) (Eq. (SourceF), M_1F = v S)."""
    lat = spec["lattice"]
    E, _, _ = O.lattice_info(lat)
    dim = O.DIMS[lat]
    n = list(spec["n"]) + [1] * (3 - len(spec["n"]))
    N = n[0] * n[1] * n[2]
    eq = spec["eq"]
    a = [F(x) for x in spec["a"]]
    ah = [F(x) for x in spec.get("ah", (0, 0, 0))]
    three = spec.get("levels", 2) == 3
    nf = O.nfields(spec)
    rho0 = F(spec.get("rho0", 0.0))
    dt, dx = F(spec.get("dt", 1.0)), F(spec.get("dx", 1.0))
    d = F(1, 3)
    if eq == "lcde":
        _, ubar, _ = O.tables(spec)
        ub = [F(float(v)) for v in ubar]
        w = None
    else:
        w = exact_weights(lat)

    def edf_at(lev, i):
        if eq == "lcde":
            return [u * lev[0][i] for u in ub]
        m = [lev[f][i] for f in range(nf)]
        if eq == "burgers":
            B = [m[0] * m[0] * dt / dx / 2] * dim
            return exact_edf(lat, E, w, m[0], B, [[F(0)] * dim for _ in range(dim)])
        rho = rho0 + m[0]
        B = m[1:]
        Cm = [[B[x] * B[y] / rho for y in range(dim)] for x in range(dim)]
        return exact_edf(lat, E, w, m[0], B, Cm)

    G = [edf_at(cur, i) for i in range(N)]
    H = [edf_at(prev, i) for i in range(N)] if three else None

    def nbr(i, j, k):
        x, y, z = i % n[0], (i // n[0]) % n[1], i // (n[0] * n[1])
        x = (x + k * E[j][0]) % n[0]
        y = (y + k * E[j][1]) % n[1]
        z = (z + k * E[j][2]) % n[2]
        return (z * n[1] + y) * n[0] + x

    if src is not None:
        wq = exact_weights(lat)
        vh = [F(float(v)) * dt / dx for v in list(src["v"]) + [0.0] * (3 - len(src["v"]))]
        St = [F(float(v)) for v in src["S_t"]]
        Sm = [F(float(v)) for v in src["S_m"]]
        bk = [F(float(v)) for v in src["b"]]
        bhk = [F(float(v)) for v in src["bh"]]

    out = [[F(0)] * N for _ in range(len(E))]
    for i in range(N):
        for j in range(len(E)):
            t = sum(a[k + 1] * G[nbr(i, j, k)][j] for k in (-1, 0, 1))
            if three:
                t += sum(ah[k + 1] * H[nbr(i, j, k)][j] for k in (-1, 0, 1))
            if src is not None:
                ev = sum(int(E[j][q]) * vh[q] for q in range(dim)) / d
                s = F(0)
                for k in (-1, 0, 1):
                    y = nbr(i, j, k)
                    s += bk[k + 1] * wq[j] * (St[y] + ev * St[y])
                    s += bhk[k + 1] * wq[j] * (Sm[y] + ev * Sm[y])
                t += dt * s
            out[j][i] = t
    return out


POP_CASES = [
    dict(lattice="D1Q3", eq="burgers", n=(5,), dx=0.25, dt=0.0625, a=(0.75, 0.25, -0.25)),
    dict(lattice="D2Q9", eq="burgers", n=(3, 3), dx=0.5, dt=0.125, a=(0.8, -0.6, -0.2)),
    dict(lattice="D2Q9", eq="burgers", n=(4, 3), dx=0.5, dt=0.125, a=(1.0, 0.0, 0.0),
         levels=3, ah=(0.125, 0.0, -0.125)),
    dict(lattice="D2Q5", eq="burgers", n=(4, 3), dx=0.5, dt=0.125, a=(0.6, -0.3, -0.1),
         levels=3, ah=(0.0, 0.0, -0.2)),
    dict(lattice="D2Q9", eq="nse", n=(4, 3), rho0=0.0, a=(1.0, 0.0, 0.0)),
    dict(lattice="D2Q9", eq="nse", n=(3, 4), rho0=1.0, a=(0.9, 0.2, -0.1)),
    dict(lattice="D3Q19", eq="nse", n=(3, 3, 2), rho0=1.0, a=(1.0, 0.0, -0.25)),
]


@pytest.mark.parametrize("spec", POP_CASES, ids=lambda s: "%s-%s-%s-L%d" % (
    s["lattice"], s["eq"], "x".join(map(str, s["n"])), s.get("levels", 2)))
def test_mesofd_populations_rational(spec):
    rng = np.random.default_rng(23)
    nf = O.nfields(spec)
    cur, prev = rand_state(spec, rng), rand_state(spec, rng)
    pop = O.init_populations(spec, cur)
    # the step reads the EDF of the moments of `pop` (rounded sums of pop)
    mom = O.moments(spec, pop)
    exact = exact_populations(spec, to_fields(mom, nf), to_fields(prev, nf))
    new, _ = O.mesofd_step(spec, pop, prev)
    N = O.npoints(spec)
    scale = max(abs(float(v)) for row in exact for v in row)
    for j, row in enumerate(exact):
        ex = np.array([float(v) for v in row])
        err = np.abs(new[j * N:(j + 1) * N] - ex).max()
        assert err <= 64 * EPS * scale, "direction %d: %g" % (j, err)


SRC_CASES = [
    dict(lattice="D2Q9", eq="lcde", n=(4, 3), u=(0.1, 0.1), K=[[0.01, 0.0], [0.0, 0.01]],
         lambda_bar=1, dx=0.25, dt=0.25 * 0.25 / 0.06 / 16, a=(1.0, 0.0, 0.0)),
    dict(lattice="D2Q9", eq="lcde", n=(3, 4), u=(0.05, -0.03), K=[[0.02, 0.005], [0.005, 0.01]],
         lambda_bar=1, dx=0.125, dt=0.125 ** 2 * 0.5, a=(-0.125, 0.25, 0.875), levels=3,
         ah=(0.125, -0.25, 0.125)),
    dict(lattice="D1Q3", eq="lcde", n=(6,), u=(0.2,), K=[[0.05]], dx=0.1, dt=0.04,
         a=(0.75, -0.5, 0.75)),
]


@pytest.mark.parametrize("spec", SRC_CASES, ids=["d2q9-2l", "d2q9-3l", "d1q3-2l"])
def test_mesofd_source_populations_rational(spec):
    rng = np.random.default_rng(29)
    N = O.npoints(spec)
    cur, prev = rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)
    src = dict(b=(1.5, 0.25, -0.125), bh=(-0.5, 0.0, 0.375), v=spec["u"],
               S_t=rng.uniform(-1, 1, N), S_m=rng.uniform(-1, 1, N))
    pop = O.init_populations(spec, cur)
    mom = O.moments(spec, pop)
    exact = exact_populations(spec, to_fields(mom, 1), to_fields(prev, 1), src)
    new, _ = O.mesofd_step(spec, pop, prev, src=src)
    scale = max(abs(float(v)) for row in exact for v in row)
    for j, row in enumerate(exact):
        ex = np.array([float(v) for v in row])
        err = np.abs(new[j * N:(j + 1) * N] - ex).max()
        assert err <= 64 * EPS * scale, "direction %d: %g" % (j, err)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_compensated_sum_against_exact(seed):
    """Neumaier summation: |s - S| <= eps |S| + 2 n^2 eps^2 sum |v| (the
    compensated-summation bound); the inputs cancel to O(1) from terms of
    1e16, where a plain left-to-right sum loses every digit."""
    rng = np.random.default_rng(seed)
    big = rng.uniform(-1e16, 1e16, 500)
    small = rng.uniform(-1.0, 1.0, 1000)
    v = np.concatenate([big, small, -big])
    rng.shuffle(v)
    exact = sum(F(float(x)) for x in v)
    s = O.csum(v)
    n = v.size
    bound = EPS * abs(float(exact)) + 2 * n * n * EPS * EPS * float(np.abs(v).sum())
    assert abs(F(s) - exact) <= F(bound)
    naive = 0.0
    for x in v:
        naive += float(x)
    assert abs(F(naive) - exact) > F(bound)  # the input really cancels
