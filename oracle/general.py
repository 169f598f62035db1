"""The MMFD scheme of Eq. (2-2-1) with any stencil reach m and any number n
of time levels: for the linear CDE (a linear EDF) on any lattice of
Appendix A (rD3Q27 included), square or rectangular, and for Burgers'
equation and the NSE (the nonlinear EDFs; the functions at the end).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Coefficients a[l][k + m] for level t - l dt (l = 0 .. n - 1) and offset
k = -m .. m.  Two forms, written independently:

* literal (the population sum of Eq. (2-1) with the moments of Eq. (2-2)):
  phi(x, t + dt) = sum_j sum_l sum_k a[l][k] f^eq_j(x + k e_j, t - l dt),
  f^eq_j = ubar_j phi (the linear EDF of Eq. (TforMMFD-0));
* central (Eq. (2-2-1)): per opposite pair p and k = 1 .. m,
  a+ = a[l][k] + a[l][-k], a- = a[l][k] - a[l][-k],
  phi' = sum_l A_l phi_l + sum_l sum_p sum_k [a+ ubp_p D2_{p,k} phi_l + a- ubm_p D1_{p,k} phi_l],
  A_l = sum_k a[l][k], D2_{p,k} g = (g(x + k e_p) - g) + (g(x - k e_p) - g),
  D1_{p,k} g = g(x + k e_p) - g(x - k e_p);
  one rounding per operation in the order written (levels, then pairs in
  lattice order, then k), which the GPU kernel follows.

The EDF's diffusion tensor takes the scheme's own moments of Eq. (4-2-00a)
with the new level at q = 0: A10 = sum_l -(l + 1) A_l and
A22 = (1/2) sum_l sum_k k^2 a[l][k], ratio = -A10 / A22.
"""
from __future__ import annotations

import numpy as np

from oracle import native as O


def moments(a):
    """(A00, A10, A11, A22) of the coefficient table a[l][k + m]."""
    a = np.asarray(a, dtype=np.float64)
    n, w = a.shape
    m = (w - 1) // 2
    A00 = 0.0
    A10 = 0.0
    A11 = 0.0
    A22 = 0.0
    for l in range(n):
        for kk in range(w):
            k = kk - m
            v = float(a[l, kk])
            A00 = A00 + v
            A10 = A10 + float(-(l + 1)) * v
            A11 = A11 + float(k) * v
            A22 = A22 + 0.5 * float(k * k) * v
    return A00, A10, A11, A22


def _spec_tables(spec, a):
    """Linear-EDF tables (w, ubar, per-pair ubp, ubm) with the scheme's ratio."""
    _, A10, _, A22 = moments(a)
    s = dict(spec)
    s["eq"] = "lcde"
    s["levels"] = 2
    s["a"] = (1.0, 0.0, 0.0)
    s["ah"] = (0.0, 0.0, 0.0)
    s["ratio"] = -A10 / A22
    w, ubar, t = O.tables(s)
    return w, ubar, t["ubp"], t["ubm"]


def _lattice(spec):
    if "d0v" in spec:
        return O.lattice_info_rect(spec["lattice"], spec["d0v"])
    return O.lattice_info(spec["lattice"], float(spec.get("d0", 1.0 / 3.0)))


def _shift(g, e, k, n):
    """g(x + k e) on the periodic grid (arrays indexed [z][y][x])."""
    dim = len(n)
    shift = tuple(-k * int(e[dim - 1 - ax]) for ax in range(dim))
    return np.roll(g, shift, axis=tuple(range(dim)))


def literal_step(spec, levels, a):
    """Eq. (2-1) summed over the directions (levels[l] = phi at t - l dt)."""
    a = np.asarray(a, dtype=np.float64)
    m = (a.shape[1] - 1) // 2
    n = tuple(spec["n"])
    shape = tuple(reversed(n))
    E, _, _ = _lattice(spec)
    _, ubar, _, _ = _spec_tables(spec, a)
    out = np.zeros(shape)
    for j in range(len(ubar)):
        fj = np.zeros(shape)
        for l, phi in enumerate(levels):
            G = ubar[j] * np.asarray(phi, dtype=np.float64).reshape(shape)
            for kk in range(2 * m + 1):
                if a[l, kk] != 0.0:
                    fj = fj + a[l, kk] * _shift(G, E[j], kk - m, n)
        out = out + fj
    return out.ravel()


def central_coefficients(spec, a):
    """A[l], Cp[l][k-1][p] = a+ ubp_p, Cm[l][k-1][p] = a- ubm_p."""
    a = np.asarray(a, dtype=np.float64)
    nl, w = a.shape
    m = (w - 1) // 2
    _, _, ubp, ubm = _spec_tables(spec, a)
    A = []
    for l in range(nl):
        s = 0.0
        for kk in range(w):
            s = s + float(a[l, kk])
        A.append(s)
    Cp = np.zeros((nl, m, len(ubp)))
    Cm = np.zeros((nl, m, len(ubp)))
    for l in range(nl):
        for k in range(1, m + 1):
            ap = float(a[l, m + k]) + float(a[l, m - k])
            am = float(a[l, m + k]) - float(a[l, m - k])
            for p in range(len(ubp)):
                Cp[l, k - 1, p] = ap * float(ubp[p])
                Cm[l, k - 1, p] = am * float(ubm[p])
    return A, Cp, Cm


def mmfd_step(spec, levels, a):
    """Eq. (2-2-1) in the order of the module docstring."""
    a = np.asarray(a, dtype=np.float64)
    m = (a.shape[1] - 1) // 2
    n = tuple(spec["n"])
    shape = tuple(reversed(n))
    E, _, pairs = _lattice(spec)
    A, Cp, Cm = central_coefficients(spec, a)
    acc = np.zeros(shape)
    phis = [np.asarray(p, dtype=np.float64).reshape(shape) for p in levels]
    for l, g in enumerate(phis):
        for p, j in enumerate(pairs):
            for k in range(1, m + 1):
                gp = _shift(g, E[j], k, n)
                gm = _shift(g, E[j], -k, n)
                d2 = (gp - g) + (gm - g)
                d1 = gp - gm
                acc = acc + Cp[l, k - 1, p] * d2
                acc = acc + Cm[l, k - 1, p] * d1
    base = A[0] * phis[0]
    for l in range(1, len(phis)):
        base = base + A[l] * phis[l]
    return (base + acc).ravel()


# ------------------------------------------------ Burgers' equation and the NSE
def _nl_spec(spec):
    s = dict(spec)
    s["levels"] = 2
    s["a"] = (1.0, 0.0, 0.0)
    s["ah"] = (0.0, 0.0, 0.0)
    s.pop("ab", None)
    s.pop("abh", None)
    return s


def nonlinear_literal_step(spec, levels, a, ab=None):
    """Eq. (2-1) with the moments of Eq. (2-2) / (2-4) for Burgers' equation
    or the NSE: f_j(x) = sum_l sum_k a[l][k] f^eq_j(x + k e_j, t - l dt), the
    density (or scalar) from sum_j f_j with the set a, the momentum from
    sum_j e_j f_j with the set ab (default a).  levels[l]: the fields of
    level t - l dt (field-major)."""
    a = np.asarray(a, dtype=np.float64)
    ab = a if ab is None else np.asarray(ab, dtype=np.float64)
    m = (a.shape[1] - 1) // 2
    s = _nl_spec(spec)
    n = tuple(spec["n"])
    shape = tuple(reversed(n))
    N = int(np.prod(n))
    E, _, _ = _lattice(spec)
    dim = O.DIMS[spec["lattice"]]
    nse = spec.get("eq") == "nse"
    pops = [O.init_populations(s, np.asarray(v, dtype=np.float64)).reshape(len(E), N)
            for v in levels]
    out = [np.zeros(shape) for _ in range(1 + dim if nse else 1)]
    for j in range(len(E)):
        for f, tab in enumerate([a] + ([ab] * dim if nse else [])):
            e = 1 if f == 0 else int(E[j][f - 1])
            if e == 0:
                continue
            fj = np.zeros(shape)
            for l, P in enumerate(pops):
                G = P[j].reshape(shape)
                for kk in range(2 * m + 1):
                    if tab[l, kk] != 0.0:
                        fj = fj + tab[l, kk] * _shift(G, E[j], kk - m, n)
            out[f] = out[f] + fj if e == 1 else out[f] - fj
    return np.concatenate([o.ravel() for o in out])


def nonlinear_mmfd_step(spec, levels, a, ab=None):
    """Eq. (2-2-1) / (2-4-1) with reach m and n levels for Burgers' equation or
    the NSE, on the pair parts F+-_p of each level (orc_pair_parts):
      density / scalar: sum_l A_l phi_l + sum_l sum_p sum_k
                        [a+_lk D2_{p,k} F+_p + a-_lk D1_{p,k} F-_p]
      momentum j_a:     sum_l Ab_l j_l + sum_l sum_{p: e_pa != 0} e_pa sum_k
                        [ab+_lk D2_{p,k} F-_p + ab-_lk D1_{p,k} F+_p]
    with D2 g = (g(x + k e_p) - g) + (g(x - k e_p) - g), D1 g = g(x + k e_p)
    - g(x - k e_p), accumulated level by level, pairs in lattice order, then
    k, each product and sum rounded on its own (the GPU kernel's order)."""
    a = np.asarray(a, dtype=np.float64)
    ab = a if ab is None else np.asarray(ab, dtype=np.float64)
    nl, w = a.shape
    m = (w - 1) // 2
    s = _nl_spec(spec)
    n = tuple(spec["n"])
    shape = tuple(reversed(n))
    N = int(np.prod(n))
    E, _, pairs = _lattice(spec)
    dim = O.DIMS[spec["lattice"]]
    nse = spec.get("eq") == "nse"
    nf = 1 + dim if nse else 1

    def sums(tab):
        A, P, M = [], np.zeros((nl, m)), np.zeros((nl, m))
        for l in range(nl):
            t = 0.0
            for kk in range(w):
                t = t + float(tab[l, kk])
            A.append(t)
            for k in range(1, m + 1):
                P[l, k - 1] = float(tab[l, m + k]) + float(tab[l, m - k])
                M[l, k - 1] = float(tab[l, m + k]) - float(tab[l, m - k])
        return A, P, M

    A, ap, am = sums(a)
    Ab, abp, abm = sums(ab)
    parts = []
    flds = []
    for v in levels:
        v = np.asarray(v, dtype=np.float64)
        Fp, Fm = O.pair_parts(s, v)
        parts.append((Fp.reshape((len(pairs),) + shape), Fm.reshape((len(pairs),) + shape)))
        flds.append(v.reshape((nf,) + shape))

    def d2(g, e, k):
        return (_shift(g, e, k, n) - g) + (_shift(g, e, -k, n) - g)

    def d1(g, e, k):
        return _shift(g, e, k, n) - _shift(g, e, -k, n)

    acc = np.zeros(shape)
    for l in range(nl):
        Fp, Fm = parts[l]
        for p, j in enumerate(pairs):
            for k in range(1, m + 1):
                acc = acc + ap[l, k - 1] * d2(Fp[p], E[j], k)
                acc = acc + am[l, k - 1] * d1(Fm[p], E[j], k)
    base = A[0] * flds[0][0]
    for l in range(1, nl):
        base = base + A[l] * flds[l][0]
    out = [base + acc]
    for f in range(1, nf):
        mo = np.zeros(shape)
        for l in range(nl):
            Fp, Fm = parts[l]
            for p, j in enumerate(pairs):
                e = int(E[j][f - 1])
                if e == 0:
                    continue
                for k in range(1, m + 1):
                    t1 = abp[l, k - 1] * d2(Fm[p], E[j], k)
                    t2 = abm[l, k - 1] * d1(Fp[p], E[j], k)
                    if e == 1:
                        mo = mo + t1
                        mo = mo + t2
                    else:
                        mo = mo - t1
                        mo = mo - t2
        bj = Ab[0] * flds[0][f]
        for l in range(1, nl):
            bj = bj + Ab[l] * flds[l][f]
        out.append(bj + mo)
    return np.concatenate([o.ravel() for o in out])
