"""Pins of the oracle's nonlinear (Burgers NCDE, NSE) steps.

* Exact rational brute force: the scheme taken literally (Eqs. (2-2)/(2-3),
  (3layerMMFD-1)) with the EDF of Eq. (3-3) evaluated in exact rational
  arithmetic on tiny periodic grids; every oracle form (MMFD central form,
  MesoFD, LITERAL) must land within a few ulp of it.
* Conservation of mass and momentum on periodic grids.
"""
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import native as O

THIRD = F(1, 3)


def exact_weights(lat):
    """Appendix A weights at d0 = 1/3 in exact arithmetic."""
    d = THIRD
    if lat == "D1Q3":
        return [1 - d, d / 2, d / 2]
    if lat == "D2Q9":
        return [(1 - d) * (1 - d)] + [d * (1 - d) / 2] * 4 + [d * d / 4] * 4
    if lat == "D3Q19":
        return [1 - 3 * d + 3 * d * d] + [d * (1 - 2 * d) / 2] * 6 + [d * d / 4] * 12
    if lat == "D2Q5II":
        return [1 - d] + [d / 4] * 4
    if lat == "D3Q7":  # at d0 = 1/3 the rest weight is 0 (Remark I: rD3Q6)
        return [1 - 3 * d] + [d / 2] * 6
    if lat == "D3Q9":
        return [1 - d] + [d / 8] * 8
    raise ValueError(lat)


def exact_edf(lat, E, w, A, B, Cm):
    d = THIRD
    dim = O.DIMS[lat]
    g = []
    for j in range(len(w)):
        e = E[j]
        t = A + sum(e[a] * B[a] for a in range(dim)) / d
        for a in range(dim):
            t += Cm[a][a] * (e[a] * e[a] - d) / (d * (1 - d))
            for b in range(dim):
                if a != b:
                    t += Cm[a][b] * e[a] * e[b] / (2 * d * d)
        g.append(w[j] * t)
    return g


def exact_step(spec, cur, prev):
    """Literal scheme in rationals: returns the new moment fields (lists)."""
    lat = spec["lattice"]
    E, _, _ = O.lattice_info(lat)
    w = exact_weights(lat)
    dim = O.DIMS[lat]
    n = list(spec["n"]) + [1] * (3 - len(spec["n"]))
    N = n[0] * n[1] * n[2]
    nf = O.nfields(spec)
    eq = spec["eq"]
    a = [F(x) for x in spec["a"]]
    ah = [F(x) for x in spec.get("ah", (0, 0, 0))]
    three = spec.get("levels", 2) == 3
    rho0 = F(spec.get("rho0", 0.0))
    bh = F(spec.get("dt", 1.0)) / F(spec.get("dx", 1.0)) / 2

    def edf_at(lev, i):
        m = [lev[f][i] for f in range(nf)]
        if eq == "burgers":
            B = [m[0] * m[0] * bh] * dim
            Cm = [[F(0)] * dim for _ in range(dim)]
            return exact_edf(lat, E, w, m[0], B, Cm)
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

    out = [[F(0)] * N for _ in range(nf)]
    for i in range(N):
        for f in range(nf):
            s = F(0)
            for j in range(len(w)):
                e = 1 if f == 0 else int(E[j][f - 1])
                if e == 0:
                    continue
                t = sum(a[k + 1] * G[nbr(i, j, k)][j] for k in (-1, 0, 1))
                if three:
                    t += sum(ah[k + 1] * H[nbr(i, j, k)][j] for k in (-1, 0, 1))
                s += e * t
            out[f][i] = s
    return out


def to_fields(arr, nf):
    N = arr.size // nf
    return [[F(float(v)) for v in arr[f * N:(f + 1) * N]] for f in range(nf)]


CASES = [
    dict(lattice="D1Q3", eq="burgers", n=(5,), dx=0.25, dt=0.0625, a=(0.75, 0.25, -0.25)),
    dict(lattice="D2Q9", eq="burgers", n=(3, 3), dx=0.5, dt=0.125, a=(0.8, -0.6, -0.2)),
    dict(lattice="D2Q9", eq="burgers", n=(4, 3), dx=0.5, dt=0.125, a=(1.0, 0.0, 0.0),
         levels=3, ah=(0.125, 0.0, -0.125)),
    dict(lattice="D2Q5II", eq="burgers", n=(3, 4), dx=0.5, dt=0.125, a=(0.8, -0.6, -0.2)),
    dict(lattice="D3Q7", eq="burgers", n=(3, 2, 3), dx=0.5, dt=0.125, a=(0.75, 0.25, -0.25)),
    dict(lattice="D3Q9", eq="burgers", n=(2, 3, 3), dx=0.5, dt=0.125, a=(0.8, -0.6, -0.2)),
    dict(lattice="D2Q9", eq="nse", n=(3, 3), rho0=1.0, a=(1.0, 0.0, -0.25), ah=(0.0, 0.25, 0.0), levels=3),
    dict(lattice="D2Q9", eq="nse", n=(4, 3), rho0=0.0, a=(1.0, 0.0, 0.0)),
    dict(lattice="D3Q19", eq="nse", n=(3, 3, 2), rho0=1.0, a=(1.0, 0.0, -0.25), ah=(0.0, 0.25, 0.0), levels=3),
]


def rand_state(spec, rng):
    N = O.npoints(spec)
    if spec["eq"] == "burgers":
        return rng.uniform(-0.5, 0.5, N)
    dim = O.DIMS[spec["lattice"]]
    base = 1.0 if spec.get("rho0", 0.0) == 0.0 else 0.0
    return np.concatenate([base + rng.uniform(-0.05, 0.05, N), rng.uniform(-0.08, 0.08, dim * N)])


@pytest.mark.parametrize("spec", CASES, ids=lambda s: "%s-%s-%s-L%d" % (s["lattice"], s["eq"], "x".join(map(str, s["n"])), s.get("levels", 2)))
def test_rational_brute_force(spec):
    rng = np.random.default_rng(17)
    nf = O.nfields(spec)
    cur, prev = rand_state(spec, rng), rand_state(spec, rng)
    exact = exact_step(spec, to_fields(cur, nf), to_fields(prev, nf))
    ex = np.array([float(v) for f in exact for v in f])
    scale = np.abs(ex).max()
    tol = 64 * np.finfo(float).eps * scale
    mm = O.mmfd_step(spec, cur, prev)
    lit = O.literal_step(spec, cur, prev)
    assert np.abs(mm - ex).max() < tol
    assert np.abs(lit - ex).max() < tol
    if spec.get("levels", 2) == 2 or spec["eq"] == "burgers":
        pop = O.init_populations(spec, cur)
        newpop, _ = O.mesofd_step(spec, pop, prev)
        assert np.abs(O.moments(spec, newpop) - ex).max() < tol


@pytest.mark.parametrize("spec", CASES[6:], ids=["d2q9-nse-3l", "d2q9-nse-2l-rho", "d3q19-nse-3l"])
def test_nse_conservation(spec):
    """Summing the central-difference form over a periodic grid leaves
    sum rho and sum j changed only by A0/Ah0 weighting (P: moment identities
    after Eq. (2-1-FD1)); with prev == cur they are conserved."""
    rng = np.random.default_rng(4)
    spec = dict(spec, n=tuple(max(v, 9) for v in spec["n"]))
    nf = O.nfields(spec)
    cur = rand_state(spec, rng)
    prev = cur.copy()
    N = O.npoints(spec)
    for _ in range(20):
        prev, cur = cur, O.mmfd_step(spec, cur, prev)
    st = rand_state(spec, np.random.default_rng(4))
    for f in range(nf):
        m0 = O.csum(st[f * N:(f + 1) * N])
        m1 = O.csum(cur[f * N:(f + 1) * N])
        assert abs(m1 - m0) < 1e-12 * (1 + np.abs(st[f * N:(f + 1) * N]).sum())
