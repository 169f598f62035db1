"""Two-level theta scheme of Eq. (GCN) for the nonlinear equations
(Burgers' NCDE with beta = 1, and the NSE), solved by Picard iteration with
the Jacobi splitting of the scheme's linear part.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

With S the explicit two-level step map of Eq. (2-2-1) (``orc_mmfd_step``) and
L(x) = S(x) - A0 x its increment (per field: A0 for the density or the
scalar, Ab0 for the momentum), Eq. (GCN) reads

    phi^{n+1} = A0 phi^n + theta L(phi^n) + (1 - theta) L(phi^{n+1}).

The EDF's parts are linear in the conserved moments up to the quadratic
term: w_p phi (the scalar, or the density in F+_p) and (w_p / d0) e_p . j
(the momentum in F-_p).  Their second differences give L the own-node
coefficient -dd per field, taken over the opposite pairs p (each pair once,
in lattice order):

    scalar / density:  dd = 2 sum_p (a_1 + a_-1) w_p
    momentum j_a:      dd = 2 sum_{p: e_pa != 0} (ab_1 + ab_-1) (w_p / d0)

(e_pa^2 = 1 for every moving velocity of these lattices).  Moving it to the
left side gives, field by field,

    R       = theta S(phi^n) + (1 - theta) (A0 phi^n)
    x_{k+1} = (R + (1 - theta) ((S(x_k) - A0 x_k) + dd x_k)) / den,
    den     = 1 + (1 - theta) dd,

started from x_0 = phi^n: the residual of x_k is den (x_{k+1} - x_k), and the
solve stops after the first chunk of sweeps with
sum_f den_f^2 sum (x_k - x_{k-1})_f^2 <= tol^2 sum_f sum R_f^2 (compensated
sums per field, added in field order), or at the first chunk boundary at or
beyond the cap.  For the linear CDE the same iteration is the Jacobi
iteration of the linear theta step.  Every node's arithmetic is written out
in the order above (one rounding per operation).
"""
from __future__ import annotations

import numpy as np

from oracle import native as O


def _explicit_spec(spec):
    s = dict(spec)
    s.pop("theta", None)
    s.pop("theta_iters", None)
    s.pop("abh", None)
    s["levels"] = 2
    s["ah"] = (0.0, 0.0, 0.0)
    return s


def picard_constants(spec):
    """(A0, dd, den) of the scalar iteration (the density's for the NSE);
    pair sums in lattice pair order."""
    a = [float(v) for v in spec["a"]]
    theta = float(spec["theta"])
    th1 = 1.0 - theta
    A0 = (a[0] + a[1]) + a[2]
    ap = a[2] + a[0]
    _, w, pairs = O.lattice_info(spec["lattice"], float(spec.get("d0", 1.0 / 3.0)))
    sp = 0.0
    for j in pairs:
        sp = sp + ap * float(w[j])
    dd = 2.0 * sp
    den = 1.0 + th1 * dd
    return A0, dd, den


def picard_field_constants(spec):
    """[(A0, dd, den)] per field: the scalar's, or the NSE's density and
    momentum components (see the module docstring)."""
    first = picard_constants(spec)
    if spec.get("eq") != "nse":
        return [first]
    d0 = float(spec.get("d0", 1.0 / 3.0))
    ab = [float(v) for v in spec.get("ab", spec["a"])]
    th1 = 1.0 - float(spec["theta"])
    Ab0 = (ab[0] + ab[1]) + ab[2]
    abp = ab[2] + ab[0]
    E, w, pairs = O.lattice_info(spec["lattice"], d0)
    out = [first]
    for a in range(O.DIMS[spec["lattice"]]):
        sj = 0.0
        for j in pairs:
            if E[j][a] != 0:
                sj = sj + abp * (float(w[j]) / d0)
        dd = 2.0 * sj
        out.append((Ab0, dd, 1.0 + th1 * dd))
    return out


def theta_picard_solve(spec, cur, tol, chunk, cap):
    """One theta step of Burgers' equation (beta = 1) or of the NSE by the
    Picard-Jacobi iteration above; returns (phi^{n+1}, sweeps, converged)."""
    eq = spec.get("eq")
    if not ((eq == "burgers" and float(spec.get("beta", 1.0)) == 1.0) or eq == "nse"):
        raise ValueError("the Picard theta step is written for Burgers' equation with beta = 1 "
                         "and for the NSE")
    es = _explicit_spec(spec)
    theta = float(spec["theta"])
    th1 = 1.0 - theta
    consts = picard_field_constants(spec)
    F = len(consts)
    N = cur.size // F
    fields = [slice(f * N, (f + 1) * N) for f in range(F)]
    S0 = O.mmfd_step(es, cur)
    R = np.empty_like(cur)
    b2 = 0.0
    for sl, (A0, _, _) in zip(fields, consts):
        R[sl] = theta * S0[sl] + th1 * (A0 * cur[sl])
        b2 = b2 + O.csum(R[sl] * R[sl])
    x = cur
    k = 0
    while True:
        for _ in range(chunk):
            Sx = O.mmfd_step(es, x)
            nxt = np.empty_like(x)
            for sl, (A0, dd, den) in zip(fields, consts):
                t = (Sx[sl] - A0 * x[sl]) + dd * x[sl]
                nxt[sl] = (R[sl] + th1 * t) * (1.0 / den)
            prev, x = x, nxt
            k += 1
        lhs = 0.0
        for sl, (_, _, den) in zip(fields, consts):
            d = x[sl] - prev[sl]
            lhs = lhs + den * den * O.csum(d * d)
        conv = lhs <= tol * tol * b2
        if conv or k >= cap:
            return x, k, bool(conv)


def theta_exact_periodic(spec, cur):
    """The linear CDE's theta step of Eq. (GCN) solved exactly on a periodic
    grid: (I - (1 - theta) L) x = R with R = theta S(phi) + (1 - theta) A0 phi
    (S the explicit step, ``orc_mmfd_step``) and L = S - A0 I, whose stencil
    sum_p [Cp_p (x(+e_p) - 2 x + x(-e_p)) + Cm_p (x(+e_p) - x(-e_p))] is the
    same at every node, so the discrete Fourier transform diagonalises it:
    x^(k) = R^(k) / (1 - (1 - theta) sum_p [Cp_p (2 cos(k.e_p) - 2)
                                            + Cm_p 2 i sin(k.e_p)]).
    (numpy's transform: a shift by +e multiplies mode k by exp(i k.e).)"""
    if spec.get("eq", "lcde") != "lcde":
        raise ValueError("the exact periodic theta step is the linear CDE's")
    es = _explicit_spec(spec)
    theta = float(spec["theta"])
    th1 = 1.0 - theta
    a = [float(v) for v in spec["a"]]
    A0 = (a[0] + a[1]) + a[2]
    S = O.mmfd_step(es, cur)
    R = theta * S + th1 * (A0 * cur)
    _, _, t = O.tables(es)
    E, _, pairs = O.lattice_info(spec["lattice"], float(spec.get("d0", 1.0 / 3.0)))
    n = list(spec["n"])
    dims = len(n)
    shape = tuple(reversed(n))  # x fastest
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(m) for m in reversed(n)], indexing="ij")
    # ks[d] is the angle per node along axis (dims - 1 - d) of the array
    sym = np.zeros(shape, dtype=np.complex128)
    for p, j in enumerate(pairs):
        ang = np.zeros(shape)
        for ax in range(dims):
            ang = ang + float(E[j][ax]) * ks[dims - 1 - ax]
        sym = sym + float(t["Cp"][p]) * (2 * np.cos(ang) - 2) + float(t["Cm"][p]) * (2j * np.sin(ang))
    Ahat = 1.0 - th1 * sym
    x = np.fft.ifftn(np.fft.fftn(R.reshape(shape)) / Ahat)
    return x.real.ravel(), R
