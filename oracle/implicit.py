"""Two-level theta scheme of Eq. (GCN) for the nonlinear scalar equation
(Burgers' NCDE, beta = 1), solved by Picard iteration with the Jacobi
splitting of the scheme's linear even part.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

With S the explicit two-level step map of Eq. (2-2-1) (``orc_mmfd_step``) and
L(x) = S(x) - A0 x its increment, Eq. (GCN) reads

    phi^{n+1} = A0 phi^n + theta L(phi^n) + (1 - theta) L(phi^{n+1}).

The even EDF part of Burgers' equation, w_j phi, is linear in phi, so L has
the diagonal -2 sum_p Cp_p with Cp_p = (a_1 + a_-1) w_p over the opposite
pairs p (each pair once).  Moving it to the left side gives the iteration

    R       = theta S(phi^n) + (1 - theta) (A0 phi^n)
    x_{k+1} = (R + (1 - theta) ((S(x_k) - A0 x_k) + dd x_k)) / den,
    dd      = 2 sum_p Cp_p,   den = 1 + (1 - theta) dd,

started from x_0 = phi^n: the residual of x_k is den (x_{k+1} - x_k), and the
solve stops after the first chunk of sweeps with
den^2 sum (x_k - x_{k-1})^2 <= tol^2 sum R^2 (compensated sums), or at the
first chunk boundary at or beyond the cap.  For the linear CDE the same
iteration is the Jacobi iteration of the linear theta step.  Every node's
arithmetic is written out in the order above (one rounding per operation).
"""
from __future__ import annotations

import numpy as np

from oracle import native as O


def _explicit_spec(spec):
    s = dict(spec)
    s.pop("theta", None)
    s.pop("theta_iters", None)
    s["levels"] = 2
    s["ah"] = (0.0, 0.0, 0.0)
    return s


def picard_constants(spec):
    """(A0, dd, den) of the iteration; pair sums in lattice pair order."""
    a = [float(v) for v in spec["a"]]
    theta = float(spec["theta"])
    th1 = 1.0 - theta
    A0 = (a[0] + a[1]) + a[2]
    ap = a[2] + a[0]
    _, w, pairs = O.lattice_info(spec["lattice"])
    sp = 0.0
    for j in pairs:
        sp = sp + ap * float(w[j])
    dd = 2.0 * sp
    den = 1.0 + th1 * dd
    return A0, dd, den


def theta_picard_solve(spec, cur, tol, chunk, cap):
    """One theta step of Burgers' equation (beta = 1) by the Picard-Jacobi
    iteration above; returns (phi^{n+1}, sweeps, converged)."""
    if spec.get("eq") != "burgers" or float(spec.get("beta", 1.0)) != 1.0:
        raise ValueError("the Picard theta step is written for Burgers' equation with beta = 1")
    es = _explicit_spec(spec)
    theta = float(spec["theta"])
    th1 = 1.0 - theta
    A0, dd, den = picard_constants(spec)
    inv_den = 1.0 / den
    S0 = O.mmfd_step(es, cur)
    R = theta * S0 + th1 * (A0 * cur)
    b2 = O.csum(R * R)
    x = cur
    k = 0
    while True:
        for _ in range(chunk):
            Sx = O.mmfd_step(es, x)
            t = (Sx - A0 * x) + dd * x
            nxt = (R + th1 * t) * inv_den
            prev, x = x, nxt
            k += 1
        d = x - prev
        conv = den * den * O.csum(d * d) <= tol * tol * b2
        if conv or k >= cap:
            return x, k, bool(conv)
