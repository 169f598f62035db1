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
