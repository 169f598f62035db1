"""Pins of the oracle's lattice tables and EDF: the printed D2Q9 weights,
the lattice moment identities of Appendix A, the EDF moment identities of
Eq. (3-5), and the reduction to the textbook LBGK equilibrium at d0 = 1/3."""
import json
import os
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import native as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_values.json")))
LATS = ["D1Q3", "D2Q5", "D2Q9", "D3Q19", "D2Q5II", "D3Q7", "D3Q9", "D3Q27"]
# Appendix A's ranges of d0 with every weight positive
D0_MAX = {"D1Q3": 1.0, "D2Q5": 0.5, "D2Q9": 1.0, "D3Q19": 0.5, "D2Q5II": 1.0, "D3Q7": 1.0 / 3.0,
          "D3Q9": 1.0, "D3Q27": 1.0}


def test_d2q9_weights_printed():
    _, w, _ = O.lattice_info("D2Q9", 1.0 / 3.0)
    want = [float(F(x)) for x in GOLD["d2q9_weights_d0_third"]["w"]]
    assert np.allclose(w, want, rtol=1e-15, atol=0)  # d0 = 1/3 is inexact: a few ulp


def test_d3q27_weights_d0_third():
    """rD3Q27 at d0 = 1/3: the product of the 1D weights 2/3, 1/6, 1/6 per
    axis: 8/27 (rest), 2/27 (axes), 1/54 (edges), 1/216 (corners)."""
    E, w, pairs = O.lattice_info("D3Q27", 1.0 / 3.0)
    nz = np.abs(E).sum(1)
    want = np.choose(nz, [8 / 27, 2 / 27, 1 / 54, 1 / 216])
    assert np.allclose(w, want, rtol=1e-15, atol=0)
    assert len(pairs) == 13 and sorted(np.bincount(nz)) == [1, 6, 8, 12]


def test_d3q19_weights_d0_third():
    _, w, _ = O.lattice_info("D3Q19", 1.0 / 3.0)
    want = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    assert np.allclose(w, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("d0", [1.0 / 3.0, 0.25, 0.4])
def test_lattice_moments(lat, d0):
    if d0 >= D0_MAX[lat]:
        pytest.skip("d0 outside the lattice's range in Appendix A")
    E, w, pairs = O.lattice_info(lat, d0)
    dim = O.DIMS[lat]
    b = len(w)
    assert len({tuple(e) for e in E}) == b  # distinct velocities
    assert np.all(w > 0)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose((w[:, None] * E).sum(0), 0, atol=1e-16)
    M2 = np.einsum("j,ja,jb->ab", w, E, E)
    assert np.allclose(M2[:dim, :dim], d0 * np.eye(dim), atol=1e-15)
    # opposite pairs: every non-rest direction appears once as e or -e
    reps = {tuple(E[j]) for j in pairs}
    assert len(pairs) == (b - 1) // 2
    for j in range(1, b):
        assert (tuple(E[j]) in reps) != (tuple(-E[j]) in reps)


def _rand_args(lat, rng):
    dim = O.DIMS[lat]
    A = rng.uniform(0.5, 1.5)
    B = rng.uniform(-0.3, 0.3, dim)
    Cm = rng.uniform(-0.2, 0.2, (dim, dim))
    Cm = 0.5 * (Cm + Cm.T)
    if lat == "D1Q3":
        Cm = np.diag(np.diag(Cm))
    if lat in ("D2Q5", "D3Q7", "D2Q5II", "D3Q9"):
        # rD2Q5I and rD3Q7 have no e_a^2 e_b^2 moment, rD2Q5II and rD3Q9 only
        # the value d0 for it (not d0^2): the quadratic part of Eq. (3-3)
        # meets the second-moment identity of Eq. (3-5) only for C = 0
        Cm = np.zeros((dim, dim))
    return A, B, Cm


@pytest.mark.parametrize("lat", LATS)
def test_edf_moment_identities(lat):
    """Eq. (3-5): sum g = A, sum e g = B, sum e e g = A d0 I + C (lattice units)."""
    rng = np.random.default_rng(11)
    E, w, _ = O.lattice_info(lat)
    dim = O.DIMS[lat]
    d0 = 1.0 / 3.0
    for _ in range(20):
        A, B, Cm = _rand_args(lat, rng)
        g = O.edf(lat, d0, A, B, Cm)
        Ed = E[:, :dim]
        assert abs(g.sum() - A) < 1e-14
        assert np.allclose(Ed.T @ g, B, atol=1e-14)
        M2 = np.einsum("j,ja,jb->ab", g, Ed, Ed)
        assert np.allclose(M2, A * d0 * np.eye(dim) + Cm, atol=1e-14)


def test_d2q5_quadratic_term_cross_talk():
    """On rD2Q5I a diagonal C_yy leaks into the xx second moment by
    -d0/(1-d0) C_yy: the reading recorded for this lattice."""
    d0 = 1.0 / 3.0
    E, w, _ = O.lattice_info("D2Q5", d0)
    g = O.edf("D2Q5", d0, 0.0, [0.0, 0.0], np.diag([0.0, 0.1]))
    M2 = np.einsum("j,ja,jb->ab", g, E[:, :2], E[:, :2])
    assert abs(M2[0, 0] - (-d0 / (1 - d0) * 0.1)) < 1e-15
    assert abs(M2[1, 1] - 0.1) < 1e-15


def test_corner_lattice_quadratic_term():
    """On rD2Q5II (and rD3Q9) every moving velocity has e_a^2 = 1, so a
    diagonal C reaches each diagonal second moment through its trace, and an
    off-diagonal C_xy comes back divided by d0: the reading recorded for
    these lattices (they serve equations with C = 0)."""
    d0 = 0.25
    for lat, dim in (("D2Q5II", 2), ("D3Q9", 3)):
        E, w, _ = O.lattice_info(lat, d0)
        Ed = E[:, :dim]
        Cd = np.diag(np.arange(1, dim + 1) * 0.01)
        g = O.edf(lat, d0, 0.0, np.zeros(dim), Cd)
        M2 = np.einsum("j,ja,jb->ab", g, Ed, Ed)
        assert np.allclose(np.diag(M2), np.trace(Cd), atol=1e-15)
        Co = np.zeros((dim, dim))
        Co[0, 1] = Co[1, 0] = 0.02
        g = O.edf(lat, d0, 0.0, np.zeros(dim), Co)
        M2 = np.einsum("j,ja,jb->ab", g, Ed, Ed)
        assert abs(M2[0, 1] - 0.02 / d0) < 1e-15


def test_d3q7_weights_and_pairs():
    """rD3Q7: w0 = 1 - 3 d0, w_axis = d0 / 2; three opposite pairs along the
    axes.  rD3Q9: w0 = 1 - d0, w_corner = d0 / 8; four corner pairs."""
    d0 = 0.25
    E, w, pairs = O.lattice_info("D3Q7", d0)
    assert np.allclose(w, [1 - 3 * d0] + [d0 / 2] * 6, rtol=0, atol=1e-16)
    assert sorted(tuple(E[j]) for j in pairs) == [(0, 0, 1), (0, 1, 0), (1, 0, 0)]
    E, w, pairs = O.lattice_info("D3Q9", d0)
    assert np.allclose(w, [1 - d0] + [d0 / 8] * 8, rtol=0, atol=1e-16)
    assert len(pairs) == 4 and all(np.abs(E[j]).sum() == 3 for j in pairs)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
def test_edf_third_moment(lat):
    """Eq. (3-7) with delta^(4) = c_s^2 (c^2 - 3 c_s^2) = 0 at d0 = 1/3:
    sum e_a e_b e_c g = d0 (delta_ab B_c + delta_ac B_b + delta_bc B_a)."""
    rng = np.random.default_rng(5)
    E, w, _ = O.lattice_info(lat)
    dim = O.DIMS[lat]
    Ed = E[:, :dim].astype(float)
    I = np.eye(dim)
    for _ in range(10):
        A, B, Cm = _rand_args(lat, rng)
        g = O.edf(lat, 1.0 / 3.0, A, B, Cm)
        M3 = np.einsum("j,ja,jb,jc->abc", g, Ed, Ed, Ed)
        want = (np.einsum("ab,c->abc", I, B) + np.einsum("ac,b->abc", I, B)
                + np.einsum("bc,a->abc", I, B)) / 3.0
        assert np.allclose(M3, want, atol=1e-14)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
def test_nse_edf_is_textbook_lbgk(lat):
    """Eq. (NSEfeq) at d0 = 1/3 equals w rho (1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u)."""
    rng = np.random.default_rng(2)
    E, w, _ = O.lattice_info(lat)
    dim = O.DIMS[lat]
    Ed = E[:, :dim]
    for _ in range(10):
        rho = rng.uniform(0.8, 1.2)
        u = rng.uniform(-0.1, 0.1, dim)
        g = O.edf(lat, 1.0 / 3.0, rho, rho * u, rho * np.outer(u, u))
        eu = Ed @ u
        want = w * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * u @ u)
        assert np.allclose(g, want, rtol=1e-14, atol=1e-16)
