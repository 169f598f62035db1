"""Pins of the oracle's source term (the b terms of Eq. (2-1) /
(3layerMMFD-1) with F_j of Eq. (SourceF), M_1F = v S), linear CDE.

* the MMFD form (pair parts of F, Eq. (2-2-1) with its b terms) equals the
  literal sum over directions and k to round-off, on every lattice, and the
  moments of the MesoFD step with the source (each population with its own
  direction's b terms) equal it too;
* its Fourier symbol: the source part of a step multiplies each mode of S
  by dt sum_j w_j (1 + e_j.vh/d0) sum_k b_k exp(i k xi.e_j);
* conservation on a periodic grid: the source adds dt (B0 sum S(t) +
  Bh0 sum S(t - dt));
* special case b = (0, 1, 0): the step adds exactly dt S;
* Example 1 (isotropic CDE with the source R, Cases 1-3): second-order
  convergence to the analytic solution in the diffusive scaling of the
  example (N_t = 0.06 N_x^2).
"""
import math

import numpy as np
import pytest

import mfd_inputs as I
from oracle import native as O
from oracle import scheme as S

LATS = ["D1Q3", "D2Q5", "D2Q9", "D3Q19"]
SCHEMES = {
    "srt": ((1, 0, 0), (0, 0, 0)),
    "ex1_case2": ((7 / 8, 1 / 4, -1 / 8), (1 / 8, -1 / 4, 1 / 8)),
    "ex1_case3": ((7 / 8, 0, 1 / 8), (1 / 8, 0, -1 / 8)),
}


def _spec(lat, name, seed):
    case = I.random_linear_case(O.DIMS[lat], seed=seed)
    a, ah = SCHEMES[name]
    K = case["K"]
    if lat == "D2Q5":  # an isotropic K keeps the rD2Q5 EDF's C = 0
        K = (np.eye(2) * 0.02).tolist()
    spec = dict(lattice=lat, n=case["n"], dx=case["dx"], dt=case["dt"], u=case["u"], K=K,
                lambda_bar=0 if lat == "D2Q5" else 1, a=a, ah=ah, levels=3 if any(ah) else 2)
    return spec, case


def _source(spec, rng):
    N = O.npoints(spec)
    d = O.DIMS[spec["lattice"]]
    return dict(b=tuple(rng.uniform(-1, 2, 3)), bh=tuple(rng.uniform(-1, 1, 3)),
                v=tuple(rng.uniform(-0.5, 0.5, d)), S_t=rng.standard_normal(N),
                S_m=rng.standard_normal(N))


@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("name", list(SCHEMES))
def test_source_forms_agree(lat, name):
    spec, case = _spec(lat, name, seed=31)
    rng = np.random.default_rng(32)
    src = _source(spec, rng)
    cur, prev = case["phi0"], case["phim"]
    mm = O.mmfd_step(spec, cur, prev, src)
    lit = O.literal_step(spec, cur, prev, src)
    scale = np.abs(cur).max() + np.abs(prev).max() + spec["dt"] * (
        np.abs(src["S_t"]).max() + np.abs(src["S_m"]).max())
    assert np.abs(mm - lit).max() < 1e-13 * scale


@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("name", list(SCHEMES))
def test_source_mesofd_moments_equal_mmfd(lat, name):
    """MesoFD with the source (each population gets dt times its direction's
    b terms): the moments of the new populations equal the MMFD step with the
    source to round-off, and the populations sum to them."""
    spec, case = _spec(lat, name, seed=39)
    rng = np.random.default_rng(40)
    src = _source(spec, rng)
    cur, prev = case["phi0"], case["phim"]
    pop = O.init_populations(spec, cur)
    newpop, mom_cur = O.mesofd_step(spec, pop, prev, src)
    meso = O.moments(spec, newpop)
    mm = O.mmfd_step(spec, cur, prev, src)
    scale = np.abs(cur).max() + np.abs(prev).max() + spec["dt"] * (
        np.abs(src["S_t"]).max() + np.abs(src["S_m"]).max())
    assert np.abs(meso - mm).max() < 1e-13 * scale
    assert np.abs(mom_cur - cur).max() < 1e-14 * scale
    # without the source the same call is the plain MesoFD step
    plain, _ = O.mesofd_step(spec, pop, prev)
    zero = dict(src, b=(0.0, 0.0, 0.0), bh=(0.0, 0.0, 0.0))
    assert np.array_equal(O.mesofd_step(spec, pop, prev, zero)[0], plain)


@pytest.mark.parametrize("lat", LATS)
def test_source_fourier_symbol(lat):
    spec, case = _spec(lat, "ex1_case3", seed=33)
    rng = np.random.default_rng(34)
    src = _source(spec, rng)
    cur, prev = case["phi0"], case["phim"]
    part = O.mmfd_step(spec, cur, prev, src) - O.mmfd_step(spec, cur, prev)
    E, w, _ = O.lattice_info(lat)
    n = spec["n"]
    d = len(n)
    vh = np.zeros(3)
    vh[:d] = np.array(src["v"]) * spec["dt"] / spec["dx"]
    shape = tuple(reversed(n))
    # mode numbers along x, y, z of the field-major (z, y, x) array
    ks = np.meshgrid(*[np.fft.fftfreq(m) * 2 * np.pi for m in reversed(n)], indexing="ij")
    kx = [ks[d - 1 - a] for a in range(d)]
    sym_t = np.zeros(shape, dtype=complex)
    sym_m = np.zeros(shape, dtype=complex)
    for j in range(len(w)):
        ph = sum(E[j][a] * kx[a] for a in range(d))
        fac = w[j] * (1.0 + float(np.dot(E[j], vh)) * 3.0)
        for k, bk, bhk in zip((-1, 0, 1), src["b"], src["bh"]):
            sym_t += fac * bk * np.exp(1j * k * ph)
            sym_m += fac * bhk * np.exp(1j * k * ph)
    want = spec["dt"] * (sym_t * np.fft.fftn(src["S_t"].reshape(shape)) +
                         sym_m * np.fft.fftn(src["S_m"].reshape(shape)))
    got = np.fft.fftn(part.reshape(shape))
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("lat", LATS)
def test_source_conservation(lat):
    spec, case = _spec(lat, "ex1_case2", seed=35)
    rng = np.random.default_rng(36)
    src = _source(spec, rng)
    cur, prev = case["phi0"], case["phim"]
    out = O.mmfd_step(spec, cur, prev, src)
    a, ah = spec["a"], spec["ah"]
    want = (sum(a) * O.csum(cur) + sum(ah) * O.csum(prev) +
            spec["dt"] * (sum(src["b"]) * O.csum(src["S_t"]) + sum(src["bh"]) * O.csum(src["S_m"])))
    scale = np.abs(cur).sum() + np.abs(prev).sum() + np.abs(src["S_t"]).sum() + np.abs(src["S_m"]).sum()
    assert abs(O.csum(out) - want) < 1e-13 * scale


@pytest.mark.parametrize("lat", LATS)
def test_source_plain_add(lat):
    """b = (0, 1, 0), bh = 0: the source part of the step is dt S(t) exactly."""
    spec, case = _spec(lat, "srt", seed=37)
    rng = np.random.default_rng(38)
    src = _source(spec, rng)
    src.update(b=(0.0, 1.0, 0.0), bh=(0.0, 0.0, 0.0))
    cur = case["phi0"]
    out = O.mmfd_step(spec, cur, None, src)
    assert np.array_equal(out, O.mmfd_step(spec, cur) + spec["dt"] * src["S_t"])


def example1_gre(case, nx):
    """Example 1 (u = (0.1, 0.1), kappa = 0.01, beta = 1, periodic [0, 2)^2
    with 2 N_x nodes a side, dx = 1/N_x, dt = 1/N_t, N_t = 0.06 N_x^2), GRE at
    T = 1 against phi = exp((1 - 2 pi^2 kappa) t) sin(pi (x + y)); the older
    level of the three-level cases is the analytic one at -dt."""
    a, ah = SCHEMES[{1: "srt", 2: "ex1_case2", 3: "ex1_case3"}[case]]
    nt = int(round(0.06 * nx * nx))
    dx, dt = 1.0 / nx, 1.0 / nt
    n = 2 * nx
    kap, u = 0.01, (0.1, 0.1)
    spec = dict(lattice="D2Q9", n=(n, n), dx=dx, dt=dt, u=u, K=[[kap, 0.0], [0.0, kap]],
                lambda_bar=1, a=a, ah=ah, levels=3 if any(ah) else 2)
    x = np.arange(n) * dx
    X, Y = np.meshgrid(x, x)
    lam = 1.0 - 2.0 * math.pi ** 2 * kap
    G = (np.sin(math.pi * (X + Y)) + math.pi * (u[0] + u[1]) * np.cos(math.pi * (X + Y))).ravel()
    phi = lambda t: math.exp(lam * t) * np.sin(math.pi * (X + Y)).ravel()
    cur, prev = phi(0.0), phi(-dt)
    for s in range(nt):
        src = dict(b=(1.5, 0.0, 0.0), bh=(-0.5, 0.0, 0.0), v=u,
                   S_t=math.exp(lam * (s * dt)) * G, S_m=math.exp(lam * ((s - 1) * dt)) * G)
        nxt = O.mmfd_step(spec, cur, prev if spec["levels"] == 3 else None, src)
        prev, cur = cur, nxt
    ex = phi(nt * dt)
    return np.abs(cur - ex).sum() / np.abs(ex).sum()


@pytest.mark.parametrize("case", [1, 2, 3])
def test_example1_second_order(case):
    errs = [example1_gre(case, nx) for nx in (10, 20, 40)]
    for i in range(2):
        p = math.log2(errs[i] / errs[i + 1])
        assert 1.9 < p < 2.15, errs
    assert errs[-1] < 4e-3
