"""Pins of the oracle's host-side scheme algebra against what the paper prints
(the constraint matrix and its inverse of Eq. (AX_b)/(invA), the closed form
of Eq. (X), the example coefficient sets of the numerical section) and against
the moment relations of Eq. (4-2-00)."""
import json
import os
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import scheme as S

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_values.json")))


def fr(v):
    return [F(x) for x in v]


def test_constraint_matrix_is_the_printed_one():
    M, _ = S.constraint_matrix()
    printed = [fr(r) for r in GOLD["constraint_matrix"]["A"]]
    assert M == printed


def test_printed_inverse_inverts_the_matrix():
    A = [fr(r) for r in GOLD["constraint_matrix"]["A"]]
    Minv = [[x / 2 for x in fr(r)] for r in GOLD["constraint_inverse"]["M"]]
    prod = [[sum(A[i][k] * Minv[k][j] for k in range(5)) for j in range(5)] for i in range(5)]
    assert prod == [[F(int(i == j)) for j in range(5)] for i in range(5)]


def test_solve_matches_closed_form_eq_X():
    rng = np.random.default_rng(7)
    for _ in range(50):
        a0, A10, A11, A21, A22 = (F(int(v), 8) for v in rng.integers(-16, 17, 5))
        (am1, a0_, a1), (ahm1, ah0, ah1) = S.solve_constraints(a0, A10, A11, A21, A22)
        # Eq. (X), written out from the printed vector
        X = [(-a0 + A10 + A11 + A21 + 2) / 2, (-a0 + A10 - A11 - A21 + 2) / 2,
             (-2 * a0 - 4 * A22 + 2) / 2, (a0 - A10 - A21 + 2 * A22 - 2) / 2,
             (a0 - A10 + A21 + 2 * A22 - 2) / 2]
        assert [a1, am1, ah0, ah1, ahm1] == X
        m = S.coeff_moments((am1, a0_, a1), (ahm1, ah0, ah1))
        assert m[(0, 0)] == 1 and m[(1, 0)] == A10 and m[(1, 1)] == A11
        assert m[(2, 1)] == A21 and m[(2, 2)] == A22
        # the relation stated after Eq. (4-2-00): A20 = -A10/2 - 1
        assert m[(2, 0)] == -A10 / 2 - 1


@pytest.mark.parametrize("ex", GOLD["examples"], ids=lambda e: e["name"])
def test_printed_example_coefficients(ex):
    g = {k: F(v) for k, v in ex["given"].items()}
    a, ah = S.solve_constraints(g["a0"], g["A10"], g["A11"], g["A21"], g["A22"])
    want_a, want_ah = fr(ex["a"]), fr(ex["ah"])
    if "misprint" in ex:
        # the printed ah_1 violates A00 = 1; the solve gives the sign-flipped value
        m = S.coeff_moments(want_a, want_ah)
        assert m[(0, 0)] == F(3, 4)
        want_ah[2] = -want_ah[2]
    assert list(a) == want_a and list(ah) == want_ah


def test_closed_forms_of_eq_4_2_00():
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = [F(int(v), 4) for v in rng.integers(-8, 9, 3)]
        ah = [F(int(v), 4) for v in rng.integers(-8, 9, 3)]
        m = S.coeff_moments(a, ah)
        (am1, a0, a1), (hm1, h0, h1) = a, ah
        assert m[(1, 0)] == -(h0 + h1 + hm1) - 1
        assert m[(1, 1)] == a1 - am1 + h1 - hm1
        assert m[(2, 0)] == (h0 + h1 + hm1 - 1) / 2
        assert m[(2, 1)] == -(h1 - hm1)
        assert m[(2, 2)] == (a1 + am1 + h1 + hm1) / 2


def test_presets():
    s = F(3, 5)
    # SRT tau = 1 equals the Ex.1 Case 1 set
    m = S.coeff_moments(*S.preset_srt())
    assert (m[(0, 0)], m[(1, 0)], m[(1, 1)], m[(2, 1)], m[(2, 2)]) == (1, -1, -1, 0, F(1, 2))
    # TRT: consistent, NCDE recovery A10 = A11, vanishing continuity error term
    m = S.coeff_moments(*S.preset_trt(s))
    assert m[(0, 0)] == 1 and m[(1, 0)] == m[(1, 1)] == -s
    assert m[(2, 2)] - m[(2, 1)] + m[(2, 0)] == 0
    # viscosity of TRT: (1/s - 1/2) dt c_s^2
    nu = S.viscosity(*S.preset_trt(F(2, 3)), dx=F(1), dt=F(1), d0=F(1, 3))
    assert nu == (F(3, 2) - F(1, 2)) * F(1, 3)
    # two-level family: A10 = A11 = -1, A22 = s/2 (Eq. LMMFD-2-1)
    m = S.coeff_moments(*S.preset_two_level(s))
    assert m[(0, 0)] == 1 and m[(1, 0)] == m[(1, 1)] == -1 and m[(2, 2)] == s / 2
    # one-stage simplified LB with tau: consistent
    m = S.coeff_moments(*S.preset_one_stage(F(7, 5)))
    assert m[(0, 0)] == 1 and m[(1, 0)] == m[(1, 1)] == -1


def test_s_for_round_trips():
    dx, dt, d0 = 0.01, 2e-5, 1.0 / 3.0
    s = S.trt_s_for(0.01, dx, dt, d0)
    assert abs(S.viscosity(*S.preset_trt(s), dx, dt, d0) - 0.01) < 1e-15
    s = S.two_level_s_for(0.003, dx, dt, d0)
    assert abs(S.diffusivity(*S.preset_two_level(s), dx, dt, d0) - 0.003) < 1e-15
