"""Pins of the oracle's multiple-set (TRT-type) schemes, Eq. (2-2-1b) and
Eq. (2-1b): the base terms take {a}, the second differences of the even EDF
parts the even set {ae}, the first differences of the odd parts the odd set
{ao} (at each time level).

* With every set equal the scheme is the single-set one, bit for bit (MMFD).
* With the base set equal to the even set, the MMFD form, the literal
  population sum of Eq. (2-1b) and the moments of the MesoFD step agree to
  round-off (linear CDE, Burgers, two- and three-level, 2D and 3D).
* With three different sets, one step of the linear CDE multiplies each
  Fourier mode by A0 + sum_p 2 [ae+ ubar+_p (cos xi_p - 1) + i ao- ubar-_p sin xi_p]
  (Eq. (TforMMFD-3b) with the sets of Eq. (2-2-1b)).
"""
import numpy as np
import pytest

from oracle import native as O

K2 = [[0.03, 0.004], [0.004, 0.02]]

CASES = [
    dict(lattice="D2Q9", eq="lcde", n=(11, 9), u=(0.1, -0.05), K=K2, lambda_bar=1,
         a=(0.6, 0.2, 0.2), ae=(0.55, 0.2, 0.25), ao=(0.9, 0.0, 0.1)),
    dict(lattice="D2Q9", eq="lcde", n=(10, 7), u=(0.1, -0.05), K=K2, lambda_bar=1, levels=3,
         a=(0.875, 0.0, 0.125), ah=(0.125, 0.0, -0.125), ae=(0.8, 0.1, 0.1),
         aeh=(0.1, -0.1, 0.1), ao=(0.95, 0.0, 0.05), aoh=(0.05, 0.0, -0.05)),
    dict(lattice="D2Q5", eq="burgers", n=(9, 8), dx=0.25, dt=0.05, a=(0.7, 0.1, 0.2),
         ae=(0.65, 0.1, 0.25), ao=(0.8, 0.1, 0.1)),
    dict(lattice="D3Q19", eq="lcde", n=(6, 5, 4), u=(0.05, 0.1, -0.05),
         K=[[0.02, 0, 0], [0, 0.03, 0], [0, 0, 0.025]], a=(0.6, 0.1, 0.3),
         ae=(0.5, 0.1, 0.4), ao=(0.7, 0.2, 0.1)),
]


def _state(spec, rng):
    N = O.npoints(spec)
    return rng.uniform(-0.5, 0.5, N)


@pytest.mark.parametrize("spec", CASES, ids=["d2q9-2l", "d2q9-3l", "d2q5-burgers", "d3q19"])
def test_equal_sets_are_the_single_set_scheme(spec):
    single = {k: v for k, v in spec.items() if k not in ("ae", "aeh", "ao", "aoh")}
    multi = dict(single, ae=single["a"], ao=single["a"], aeh=single.get("ah", (0, 0, 0)),
                 aoh=single.get("ah", (0, 0, 0)))
    rng = np.random.default_rng(1)
    cur, prev = _state(spec, rng), _state(spec, rng)
    assert np.array_equal(O.mmfd_step(multi, cur, prev), O.mmfd_step(single, cur, prev))


@pytest.mark.parametrize("spec", CASES, ids=["d2q9-2l", "d2q9-3l", "d2q5-burgers", "d3q19"])
def test_forms_agree_with_base_equal_to_even_set(spec):
    spec = dict(spec, a=spec["ae"], ah=spec.get("aeh", (0, 0, 0)))
    rng = np.random.default_rng(2)
    cur, prev = _state(spec, rng), _state(spec, rng)
    mm = O.mmfd_step(spec, cur, prev)
    lit = O.literal_step(spec, cur, prev)
    pop = O.init_populations(spec, cur)
    new, _ = O.mesofd_step(spec, pop, prev)
    mo = O.moments(spec, new)
    # the step the MesoFD form takes reads the EDF of the moments of `pop`
    mm2 = O.mmfd_step(spec, O.moments(spec, pop), prev)
    scale = np.abs(mm).max()
    assert np.abs(mm - lit).max() < 1e-14 * scale
    assert np.abs(mo - mm2).max() < 1e-14 * scale
    # and the sets really differ from the single-set scheme
    single = {k: v for k, v in spec.items() if k not in ("ae", "aeh", "ao", "aoh")}
    assert np.abs(O.mmfd_step(single, cur, prev) - mm).max() > 1e-6 * scale


def test_fourier_symbol_three_sets():
    spec = CASES[0]
    E, w, pairs = O.lattice_info("D2Q9")
    _, _, tab = O.tables(spec)
    rng = np.random.default_rng(3)
    n = spec["n"]
    phi = rng.standard_normal(n[0] * n[1])
    out = O.mmfd_step(spec, phi)
    a, ae, ao = spec["a"], spec["ae"], spec["ao"]
    ky = 2 * np.pi * np.fft.fftfreq(n[1])[:, None]
    kx = 2 * np.pi * np.fft.fftfreq(n[0])[None, :]
    lam = np.full((n[1], n[0]), float(sum(a)), dtype=complex)
    for p, j in enumerate(pairs):
        xi = E[j][0] * kx + E[j][1] * ky
        lam += 2 * ((ae[2] + ae[0]) * tab["ubp"][p] * (np.cos(xi) - 1)
                    + 1j * (ao[2] - ao[0]) * tab["ubm"][p] * np.sin(xi))
    fo = np.fft.fft2(out.reshape(n[1], n[0]))
    fi = np.fft.fft2(phi.reshape(n[1], n[0]))
    assert np.abs(fo - lam * fi).max() < 1e-12 * np.abs(fi).max()
