"""Pins of the oracle's general MMFD scheme (any stencil reach m, any number
n of time levels; oracle/general.py) for the linear CDE.

* Its two forms, the population sum of Eq. (2-1)/(2-2) and the central pair
  form of Eq. (2-2-1), written independently, agree to rounding for
  m = 1 .. 3, n = 1 .. 4, on square, rectangular and rD3Q27 lattices.
* m = 1 with one or two levels is the two-level / three-level scheme of the
  oracle's own step (orc_mmfd_step), to rounding.
* The moments of Eq. (4-2-00a) give the EDF's diffusion: with A00 = 1 and
  A11 = A10, a long Fourier mode (the other levels holding the same mode
  decayed at the physical rate) decays at K k^2 per unit time, for wide and
  multi-level schemes and on rD3Q27.
* Burgers' equation and the NSE: the population and pair-part forms agree,
  m = 1 is the oracle's own step, the NSE keeps mass and momentum, and a
  shear wave decays at the viscosity of the momentum set's own moments.
"""
import numpy as np
import pytest

from oracle import general as GN
from oracle import native as O


def _spec(lat, n, **kw):
    dim = O.DIMS[lat]
    base = dict(lattice=lat, eq="lcde", n=n, dx=1.0, dt=1.0, u=[0.05, -0.03, 0.02][:dim],
                K=(np.eye(dim) * 0.1 + 0.01 * (np.ones((dim, dim)) - np.eye(dim))).tolist(),
                lambda_bar=1)
    base.update(kw)
    return base


def _consistent(rng, m, n):
    """A random table with A00 = 1, A11 = A10 and -A10 / A22 > 0."""
    while True:
        a = rng.uniform(-0.3, 0.6, (n, 2 * m + 1))
        # A00 = 1 through a[0][m] (k = 0); A11 = A10 through a[0][m - 1] (k = -1)
        for _ in range(2):
            A00, A10, A11, A22 = GN.moments(a)
            a[0, m - 1] += (A11 - A10)  # k = -1 lowers A11 by the entry, A10 by it too
            A00, A10, A11, A22 = GN.moments(a)
            a[0, m] += 1.0 - A00
        A00, A10, A11, A22 = GN.moments(a)
        if abs(A00 - 1) < 1e-14 and abs(A11 - A10) < 1e-12 and A10 < 0 and A22 > 0.05:
            return a


CASES = [("D2Q9", (11, 9), {}), ("D2Q5", (10, 7), {}), ("D1Q3", (23,), {}),
         ("D3Q19", (7, 6, 5), {}), ("D3Q27", (7, 6, 5), {}),
         ("D2Q9", (12, 9), dict(dxv=(0.5, 2.0), d0v=(0.3, 0.45))),
         ("D3Q27", (6, 7, 5), dict(dxv=(1.0, 0.5, 2.0), d0v=(0.3, 0.4, 0.5)))]


@pytest.mark.parametrize("lat,n,kw", CASES)
@pytest.mark.parametrize("m,nl", [(1, 1), (2, 1), (3, 2), (2, 3), (1, 4)])
def test_literal_and_central_forms_agree(lat, n, kw, m, nl):
    rng = np.random.default_rng(m * 10 + nl)
    spec = _spec(lat, n, **kw)
    a = rng.uniform(-0.5, 0.8, (nl, 2 * m + 1))
    N = int(np.prod(n))
    levels = [rng.standard_normal(N) for _ in range(nl)]
    lit = GN.literal_step(spec, levels, a)
    cen = GN.mmfd_step(spec, levels, a)
    scale = max(np.abs(lit).max(), 1.0)
    assert np.allclose(cen, lit, rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("lat,n", [("D2Q9", (11, 9)), ("D3Q19", (6, 5, 4))])
def test_m1_is_the_two_and_three_level_scheme(lat, n):
    rng = np.random.default_rng(5)
    spec = _spec(lat, n)
    N = int(np.prod(n))
    phi, prev = rng.standard_normal(N), rng.standard_normal(N)
    a2 = np.array([[1.0, 0.0, 0.0]])
    got = GN.mmfd_step(spec, [phi], a2)
    want = O.mmfd_step(dict(spec, a=(1.0, 0.0, 0.0)), phi)
    assert np.allclose(got, want, rtol=0, atol=1e-14 * np.abs(want).max())
    a3 = np.array([[0.875, 0.25, -0.125], [0.125, -0.25, 0.125]])
    got = GN.mmfd_step(spec, [phi, prev], a3)
    want = O.mmfd_step(dict(spec, a=tuple(a3[0]), ah=tuple(a3[1]), levels=3), phi, prev)
    assert np.allclose(got, want, rtol=0, atol=1e-14 * np.abs(want).max())


def _rate(spec, a, axis):
    """The decay rate per unit time of a long mode along `axis` after one
    step, the older levels holding the mode decayed at the physical rate."""
    n = spec["n"]
    a = np.asarray(a)
    dim = len(n)
    idx = np.indices(tuple(reversed(n)))
    th = (2 * np.pi * idx[dim - 1 - axis] / n[axis]).ravel()
    k = 2 * np.pi / (n[axis] * spec.get("dxv", [spec["dx"]] * 3)[axis])
    K = spec["K"][axis][axis]
    dt = spec["dt"]
    xi = np.exp(-K * k * k * dt)
    out = []
    for comp in (np.cos, np.sin):
        lev = [comp(th) * xi ** (-l) for l in range(a.shape[0])]
        out.append(GN.mmfd_step(spec, lev, a))
    z = out[0] + 1j * out[1]
    e = np.exp(1j * th)
    G = np.vdot(e, z) / np.vdot(e, e)
    return -np.log(abs(G)) / dt, K * k * k


# (rD2Q5I and rD3Q7 meet the second-moment identity of Eq. (3-5) only for C = 0,
# which a scheme's own ratio does not give in general, so the lattices here
# are those with every e_a^2 e_b^2 moment)
@pytest.mark.parametrize("lat,n,axis", [("D2Q9", (256, 4), 0), ("D2Q9", (4, 256), 1),
                                        ("D3Q27", (4, 4, 256), 2)])
@pytest.mark.parametrize("m,nl", [(2, 1), (3, 1), (1, 2), (2, 2), (2, 3)])
def test_general_moments_give_the_physical_diffusion(lat, n, axis, m, nl):
    rng = np.random.default_rng(100 + m * 10 + nl)
    a = _consistent(rng, m, nl)
    dim = O.DIMS[lat]
    spec = dict(lattice=lat, eq="lcde", n=n, dx=1.0, dt=0.05, u=[0.0] * dim,
                K=(np.eye(dim) * 0.4).tolist())
    rate, want = _rate(spec, a, axis)
    assert abs(rate / want - 1) < 5e-3, (rate, want)


# ------------------------------------------------ Burgers' equation and the NSE
NL = [("D2Q9", (9, 7), "burgers"), ("D1Q3", (17,), "burgers"), ("D2Q9", (9, 7), "nse"),
      ("D3Q19", (5, 4, 4), "nse"), ("D2Q5", (8, 6), "nse")]


def _nl_state(lat, n, eq, rng, amp=0.05):
    N = int(np.prod(n))
    nf = 1 + len(n) if eq == "nse" else 1
    return amp * rng.uniform(-1, 1, nf * N)


@pytest.mark.parametrize("lat,n,eq", NL)
@pytest.mark.parametrize("m,nl", [(1, 1), (2, 1), (2, 2), (3, 3)])
def test_nonlinear_literal_and_central_forms_agree(lat, n, eq, m, nl):
    rng = np.random.default_rng(7 * m + nl)
    spec = dict(lattice=lat, eq=eq, n=n, dx=1.0, dt=1.0, rho0=1.0, beta=1.0)
    a = rng.uniform(-0.3, 0.6, (nl, 2 * m + 1))
    ab = rng.uniform(-0.3, 0.6, (nl, 2 * m + 1)) if eq == "nse" else None
    lev = [_nl_state(lat, n, eq, rng) for _ in range(nl)]
    lit = GN.nonlinear_literal_step(spec, lev, a, ab)
    cen = GN.nonlinear_mmfd_step(spec, lev, a, ab)
    assert np.allclose(cen, lit, rtol=0, atol=1e-14 * max(np.abs(lit).max(), 1.0))


@pytest.mark.parametrize("lat,n,eq", NL)
def test_nonlinear_m1_is_the_two_and_three_level_scheme(lat, n, eq):
    rng = np.random.default_rng(9)
    spec = dict(lattice=lat, eq=eq, n=n, dx=1.0, dt=1.0, rho0=1.0, beta=1.0)
    cur, prev = _nl_state(lat, n, eq, rng), _nl_state(lat, n, eq, rng)
    a2 = np.array([[0.6, 0.1, 0.3]])
    ab2 = np.array([[0.7, 0.0, 0.3]]) if eq == "nse" else None
    got = GN.nonlinear_mmfd_step(spec, [cur], a2, ab2)
    kw = dict(a=tuple(a2[0]))
    if ab2 is not None:
        kw["ab"] = tuple(ab2[0])
    want = O.mmfd_step(dict(spec, **kw), cur)
    assert np.allclose(got, want, rtol=0, atol=1e-15 * max(np.abs(want).max(), 1.0))
    a3 = np.array([[0.875, 0.25, -0.125], [0.125, -0.25, 0.125]])
    ab3 = np.array([[0.8, 0.3, -0.1], [0.1, -0.2, 0.1]]) if eq == "nse" else None
    got = GN.nonlinear_mmfd_step(spec, [cur, prev], a3, ab3)
    kw = dict(a=tuple(a3[0]), ah=tuple(a3[1]), levels=3)
    if ab3 is not None:
        kw.update(ab=tuple(ab3[0]), abh=tuple(ab3[1]))
    want = O.mmfd_step(dict(spec, **kw), cur, prev)
    assert np.allclose(got, want, rtol=0, atol=1e-15 * max(np.abs(want).max(), 1.0))


def test_nonlinear_general_nse_conserves_mass_and_momentum():
    """With A00 = Ab00 = 1 and equal levels, the totals of mass and momentum
    are kept (the differences sum to zero on a periodic grid)."""
    rng = np.random.default_rng(10)
    spec = dict(lattice="D2Q9", eq="nse", n=(12, 10), dx=1.0, dt=1.0, rho0=1.0)
    a = _consistent(rng, 2, 2)
    ab = _consistent(rng, 2, 2)
    v = _nl_state("D2Q9", (12, 10), "nse", rng)
    out = GN.nonlinear_mmfd_step(spec, [v, v], a, ab)
    N = 120
    for f in range(3):
        assert abs(out[f * N:(f + 1) * N].sum() - v[f * N:(f + 1) * N].sum()) < 1e-13


@pytest.mark.parametrize("m,nl", [(2, 1), (1, 2), (2, 2)])
def test_nonlinear_general_nse_shear_viscosity(m, nl):
    """A small shear wave j_x = U sin(k y) on rD2Q9 decays at nu k^2 with the
    viscosity of the momentum set's own moments, nu = -(Ab22 / Ab10) dt c_s^2
    (lattice units: c_s^2 = d0), the older levels holding the wave decayed at
    that rate: the moments of Eq. (4-2-00a) give the NSE's viscosity for
    wide and multi-level schemes."""
    rng = np.random.default_rng(200 + 10 * m + nl)
    ab = _consistent(rng, m, nl)
    a = _consistent(rng, m, nl)
    _, A10, _, A22 = GN.moments(ab)
    nu = -(A22 / A10) * (1.0 / 3.0)
    n = (4, 256)
    N = 4 * 256
    y = np.indices((256, 4))[0].ravel()
    k = 2 * np.pi / 256
    xi = np.exp(-nu * k * k)
    U = 1e-6
    spec = dict(lattice="D2Q9", eq="nse", n=n, dx=1.0, dt=1.0, rho0=1.0)
    lev = [np.concatenate([np.zeros(N), U * np.sin(k * y) * xi ** (-l), np.zeros(N)])
           for l in range(nl)]
    out = GN.nonlinear_mmfd_step(spec, lev, a, ab)
    jx = out[N:2 * N]
    G = (jx @ np.sin(k * y)) / (U * np.sin(k * y) @ np.sin(k * y))
    rate = -np.log(G)
    assert abs(rate / (nu * k * k) - 1) < 5e-3, (rate, nu * k * k)
