"""Host-side algebra of the EDF-based MesoFD / MMFD schemes (oracle side).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Coefficient vectors are ``(a_-1, a_0, a_1)`` for time level t and
``(ah_-1, ah_0, ah_1)`` for level t - dt, the three-level notation of
Eq. (3layer-1).  Every function works on ``fractions.Fraction`` as well as on
floats, so the exact rational pins can run through the same code.
"""
from __future__ import annotations

from fractions import Fraction
from math import comb, factorial

import numpy as np


# --------------------------------------------------------------- moments A_lm

def coeff_moments(a, ah, lmax=2):
    """A_lm of Eq. (4-2) for a scheme that produces phi(x, t+dt).

    Eq. (4-2) with level t at q = 0 and t - dt at q = -1, and the shift of
    Remark 1 (5): because the left-hand side sits at t + dt, A_l0 loses 1/l!.
    Returns a dict {(l, m): A_lm}.
    """
    terms = [(k, 0, a[k + 1]) for k in (-1, 0, 1)] + [(k, -1, ah[k + 1]) for k in (-1, 0, 1)]
    out = {}
    for l in range(lmax + 1):
        for m in range(l + 1):
            s = 0
            for k, q, v in terms:
                s = s + v * (q ** (l - m)) * (k ** m)
            val = Fraction(comb(l, m), factorial(l)) * s if isinstance(s, Fraction) else comb(l, m) / factorial(l) * s
            if m == 0 and l >= 1:
                val = val - (Fraction(1, factorial(l)) if isinstance(val, Fraction) else 1.0 / factorial(l))
            out[(l, m)] = val
    return out


def constraint_matrix():
    """The 5x5 system of Eq. (AX_b): rows are the A00, A10, A11, A21, A22
    conditions of Eq. (4-2-00a) written as linear functions of
    X = (a_1, a_-1, ah_0, ah_1, ah_-1), obtained here by evaluating
    `coeff_moments` on unit vectors (so the matrix is derived, not typed)."""
    rows = []
    unit = []
    for i in range(5):
        x = [Fraction(0)] * 5
        x[i] = Fraction(1)
        unit.append(x)
    # constant parts (a_0 = 0, X = 0)
    m0 = coeff_moments((0, 0, 0), (0, 0, 0))
    cols = []
    for x in unit:
        a = (x[1], Fraction(0), x[0])
        ah = (x[4], x[2], x[3])
        m = coeff_moments(a, ah)
        cols.append([m[(0, 0)] - m0[(0, 0)], m[(1, 0)] - m0[(1, 0)], m[(1, 1)] - m0[(1, 1)],
                     m[(2, 1)] - m0[(2, 1)], m[(2, 2)] - m0[(2, 2)]])
    for r in range(5):
        rows.append([cols[c][r] for c in range(5)])
    return rows, m0


def _solve_exact(M, rhs):
    n = len(rhs)
    A = [list(map(Fraction, M[i])) + [Fraction(rhs[i])] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [A[r][k] - f * A[c][k] for k in range(n + 1)]
    return [A[i][n] / A[i][i] for i in range(n)]


def solve_constraints(a0, A10, A11, A21, A22):
    """Coefficients from the conditions of Eq. (4-2-00a) (A00 = 1 imposed):
    returns (a, ah) with a = (a_-1, a_0, a_1), ah = (ah_-1, ah_0, ah_1).
    Exact rational Gaussian elimination of the system of Eq. (AX_b)."""
    a0, A10, A11, A21, A22 = (Fraction(v) for v in (a0, A10, A11, A21, A22))
    M, m0 = constraint_matrix()
    # A00 row: a_0 + (sum of X entries) = 1; A10 row includes the -1 shift.
    target = [Fraction(1) - a0, A10 - m0[(1, 0)], A11, A21, A22]
    X = _solve_exact(M, target)
    a1, am1, ah0, ah1, ahm1 = X
    return (am1, a0, a1), (ahm1, ah0, ah1)


# ------------------------------------------------------------------- presets

def preset_srt():
    """SRT LB with tau = 1 (first preset of the three-level family)."""
    return (1, 0, 0), (0, 0, 0)


def preset_trt(s):
    """TRT LB with s+ + s- = 2, s = s-:  a_0 = 0, a_1 = 1 - s, a_-1 = 1,
    ah_0 = -(1 - s)."""
    return (1, 0, 1 - s), (0, -(1 - s), 0)


def preset_one_stage(tau):
    """One-stage simplified LB: a_0 = 2(1 - tau), a_1 = tau - 1, a_-1 = tau."""
    return (tau, 2 * (1 - tau), tau - 1), (0, 0, 0)


def preset_two_level(s):
    """General m = 1 two-level explicit family, Eq. (LMMFD-2-2), with
    s = 2 alpha / (dt c_s^2):  a_0 = 1 - s, a_1 = (s - 1)/2, a_-1 = (s + 1)/2."""
    return ((s + 1) / 2, 1 - s, (s - 1) / 2), (0, 0, 0)


# ------------------------------------------------- PDE-coefficient mapping

def lattice_cs2(dx, dt, d0):
    return d0 * (dx / dt) ** 2


def diffusivity(a, ah, dx, dt, d0, beta=1.0):
    """alpha = -(A22 / A10) dt beta c_s^2."""
    m = coeff_moments(a, ah)
    return -(m[(2, 2)] / m[(1, 0)]) * dt * beta * lattice_cs2(dx, dt, d0)


def viscosity(ab, abh, dx, dt, d0):
    """nu = -(Abar22 / Abar10) dt c_s^2."""
    m = coeff_moments(ab, abh)
    return -(m[(2, 2)] / m[(1, 0)]) * dt * lattice_cs2(dx, dt, d0)


def two_level_s_for(alpha, dx, dt, d0, beta=1.0):
    """s of the two-level family giving diffusivity alpha."""
    return 2.0 * alpha / (dt * beta * lattice_cs2(dx, dt, d0))


def trt_s_for(nu, dx, dt, d0):
    """s of the TRT preset giving viscosity nu: nu = (1/s - 1/2) dt c_s^2."""
    return 1.0 / (nu / (dt * lattice_cs2(dx, dt, d0)) + 0.5)


# ------------------------------------------------------------------ stability

def theorem1(a, ubp, ubm):
    """Conditions (a), (b), (c) of Theorem 1 for a two-level explicit linear
    scheme with m = 1; ubp / ubm are the pair values ubar+_j / ubar-_j (each
    pair stands for j and jbar, which have equal summands)."""
    ap = a[2] + a[0]
    am = a[2] - a[0]
    terms = [ap * u for u in ubp]
    cond_a = all(t > 0 for t in terms)
    cond_b = 2 * sum(terms) <= 1
    cond_c = 2 * sum(((am * v) ** 2) / t for t, v in zip(terms, ubm) if t > 0) <= 1
    return cond_a, cond_b, cond_c


def linear_edf_bound_dt(D, u, dx, d0_w0):
    """Eq. (LMMFD-2-3) for the m = 1 two-level scheme with the linear EDF:
    |u|^2 <= 2 alpha / dt <= c_s^2 / (1 - w0).  With c_s^2 = d0 dx^2/dt^2
    this is dt <= min( d0 dx^2 / (2 D (1 - w0)), 2 D / |u|^2 ).
    d0_w0 = (d0, w0)."""
    d0, w0 = d0_w0
    u2 = float(np.dot(u, u))
    t1 = d0 * dx * dx / (2.0 * D * (1.0 - w0))
    return t1 if u2 == 0.0 else min(t1, 2.0 * D / u2)


def fourier_symbols(E, pairs, ubp, ubm, n, a, ah):
    """A_{-1}(xi), A_{-2}(xi) of Eq. (TforMMFD-3b) (three-level explicit,
    A_0 = 0) on the grid modes xi_alpha = 2 pi m / n_alpha of a periodic grid
    with n = (nx[, ny[, nz]]) nodes.  Arrays are shaped like numpy's FFT of a
    field stored [z][y][x]; each opposite pair contributes twice (j, jbar)."""
    dim = len(n)
    shape = tuple(reversed(n))
    grids = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(nn) for nn in shape], indexing="ij")
    xi_axis = [grids[dim - 1 - d] for d in range(dim)]  # xi_x, xi_y, xi_z
    A1 = np.full(shape, float(sum(a)), dtype=complex)
    A2 = np.full(shape, float(sum(ah)), dtype=complex)
    ap, am = a[2] + a[0], a[2] - a[0]
    hp, hm = ah[2] + ah[0], ah[2] - ah[0]
    for p, j in enumerate(pairs):
        xi = sum(E[j][d] * xi_axis[d] for d in range(dim))
        cm1 = np.cos(xi) - 1.0
        sn = np.sin(xi)
        A1 += 2 * (ap * ubp[p] * cm1 + 1j * am * ubm[p] * sn)
        A2 += 2 * (hp * ubp[p] * cm1 + 1j * hm * ubm[p] * sn)
    return A1, A2


def max_amplification(E, pairs, ubp, ubm, n, a, ah):
    """max over grid modes of the largest root modulus of
    lambda^2 - p1 lambda - p0 (Eq. 3-level) with p1 = A_{-1}, p0 = A_{-2};
    for two-level schemes (ah = 0) this is max |A_{-1}|."""
    p1, p0 = fourier_symbols(E, pairs, ubp, ubm, n, a, ah)
    disc = np.sqrt(p1 * p1 + 4 * p0)
    r1 = np.abs((p1 + disc) / 2)
    r2 = np.abs((p1 - disc) / 2)
    return float(np.max(np.maximum(r1, r2)))


def theorem3(p1, p0):
    """Schur-Cohn condition of Theorem 3: |p1 + conj(p1) p0| <= 1 - |p0|^2."""
    return np.abs(p1 + np.conj(p1) * p0) <= 1 - np.abs(p0) ** 2
