"""ctypes binding of the plain-C FP64 oracle (``mfd_oracle.c``).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Arrays are numpy float64, field-major ``[field][z][y][x]`` (x fastest), the
same layout for moments (``nf`` fields) and populations (``b`` fields).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mfd_oracle.c")
LIB = os.path.join(HERE, "libmfd_oracle.so")

LATTICES = {"D1Q3": 1, "D2Q5": 2, "D2Q9": 3, "D3Q19": 4, "D2Q5II": 5, "D3Q7": 6, "D3Q9": 7,
            "D3Q27": 8}
DIMS = {"D1Q3": 1, "D2Q5": 2, "D2Q9": 2, "D3Q19": 3, "D2Q5II": 2, "D3Q7": 3, "D3Q9": 3,
        "D3Q27": 3}
QS = {"D1Q3": 3, "D2Q5": 5, "D2Q9": 9, "D3Q19": 19, "D2Q5II": 5, "D3Q7": 7, "D3Q9": 9,
      "D3Q27": 27}
EQS = {"lcde": 0, "burgers": 1, "nse": 2, "wave": 3}
MAXP = 13
MAXQ = 27


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: no fast-math, no FMA contraction."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
             "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("eq", C.c_int32), ("levels", C.c_int32),
        ("lambda_bar", C.c_int32), ("he_luo", C.c_int32), ("nthreads", C.c_int32),
        ("theta_iters", C.c_int32), ("bc", C.c_int32),
        ("n", C.c_int64 * 3),
        ("d0", C.c_double), ("dx", C.c_double), ("dt", C.c_double),
        ("u", C.c_double * 3), ("K", C.c_double * 9),
        ("beta", C.c_double), ("rho0", C.c_double),
        ("a", C.c_double * 3), ("ah", C.c_double * 3),
        ("ab", C.c_double * 3), ("abh", C.c_double * 3),
        ("theta", C.c_double),
        ("bscale", C.c_double), ("bG", C.POINTER(C.c_double)),
        ("multiset", C.c_int32), ("pad2_", C.c_int32),
        ("ae", C.c_double * 3), ("aeh", C.c_double * 3),
        ("ao", C.c_double * 3), ("aoh", C.c_double * 3),
        ("rect", C.c_int32), ("pad3_", C.c_int32),
        ("d0v", C.c_double * 3), ("dxv", C.c_double * 3),
        ("ratio", C.c_double),
    ]


class Source(C.Structure):
    _fields_ = [("b", C.c_double * 3), ("bh", C.c_double * 3), ("v", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        P = C.POINTER(Params)
        D = C.POINTER(C.c_double)
        for name, args in [
            ("orc_mmfd_step", [P, D, D, D]),
            ("orc_literal_step", [P, D, D, D]),
            ("orc_init_populations", [P, D, D]),
            ("orc_moments", [P, D, D]),
            ("orc_mesofd_step", [P, D, D, D, D]),
            ("orc_theta_step", [P, D, D, D]),
            ("orc_tables", [P, D, D, D]),
            ("orc_pair_parts", [P, D, D, D]),
            ("orc_wave_start", [P, D, D, D]),
            ("orc_mmfd_source_step", [P, C.POINTER(Source), D, D, D, D, D]),
            ("orc_literal_source_step", [P, C.POINTER(Source), D, D, D, D, D]),
            ("orc_mesofd_source_step", [P, C.POINTER(Source), D, D, D, D, D, D]),
        ]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.orc_lattice_info.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_int), D,
                                       C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_lattice_info.restype = C.c_int
        L.orc_edf.argtypes = [C.c_int, C.c_double, C.c_double, D, D, D]
        L.orc_edf.restype = C.c_int
        L.orc_lattice_info_rect.argtypes = [C.c_int, D, C.POINTER(C.c_int), D,
                                            C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_lattice_info_rect.restype = C.c_int
        L.orc_edf_rect.argtypes = [C.c_int, D, C.c_double, D, D, D]
        L.orc_edf_rect.restype = C.c_int
        L.orc_theta_solve.argtypes = [P, D, D, D, C.c_double, C.c_int, C.c_int,
                                      C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_theta_solve.restype = C.c_int
        L.orc_sum.argtypes = [D, C.c_int64]
        L.orc_sum.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _triple(v, fill=0.0):
    v = list(v) + [fill] * (3 - len(v))
    return (C.c_double * 3)(*v)


def make_params(spec: dict) -> Params:
    """Build the C parameter block from a plain problem description.

    spec keys: lattice, n (tuple), d0, dx, dt, eq ('lcde'|'burgers'|'nse'),
    levels (2|3), a (k=-1,0,1), ah, ab, abh (default: a, ah), u, K (dim x dim),
    lambda_bar, beta, rho0, he_luo, theta, theta_iters, nthreads.
    """
    P = Params()
    lat = spec["lattice"]
    P.lattice = LATTICES[lat]
    P.eq = EQS[spec.get("eq", "lcde")]
    P.levels = int(spec.get("levels", 2))
    P.lambda_bar = int(spec.get("lambda_bar", 0))
    P.he_luo = int(spec.get("he_luo", 0))
    P.nthreads = int(spec.get("nthreads", 0))
    P.theta_iters = int(spec.get("theta_iters", 0))
    n = list(spec["n"]) + [1] * (3 - len(spec["n"]))
    P.n = (C.c_int64 * 3)(*n)
    P.d0 = float(spec.get("d0", 1.0 / 3.0))
    P.dx = float(spec.get("dx", 1.0))
    P.dt = float(spec.get("dt", 1.0))
    P.u = _triple([float(x) for x in spec.get("u", ())])
    Kd = np.zeros((3, 3))
    K = np.asarray(spec.get("K", np.zeros((1, 1))), dtype=np.float64)
    Kd[: K.shape[0], : K.shape[1]] = K
    P.K = (C.c_double * 9)(*Kd.ravel().tolist())
    P.beta = float(spec.get("beta", 1.0))
    P.rho0 = float(spec.get("rho0", 0.0))
    a = [float(x) for x in spec["a"]]
    ah = [float(x) for x in spec.get("ah", (0.0, 0.0, 0.0))]
    P.a = _triple(a)
    P.ah = _triple(ah)
    P.ab = _triple([float(x) for x in spec.get("ab", a)])
    P.abh = _triple([float(x) for x in spec.get("abh", ah)])
    P.theta = float(spec.get("theta", 1.0))
    P.ratio = float(spec.get("ratio", 0.0))
    if "d0v" in spec or "dxv" in spec:
        # rectangular lattice (linear CDE): d0 and spacing per axis
        d0 = float(spec.get("d0", 1.0 / 3.0))
        dx = float(spec.get("dx", 1.0))
        d0v = list(spec.get("d0v", [d0] * 3)) + [d0] * 3
        dxv = list(spec.get("dxv", [dx] * 3)) + [dx] * 3
        P.rect = 1
        P.d0v = (C.c_double * 3)(*[float(v) for v in d0v[:3]])
        P.dxv = (C.c_double * 3)(*[float(v) for v in dxv[:3]])
    if "ae" in spec or "ao" in spec:
        # multiple-set scheme, Eq. (2-2-1b): even set ae/aeh, odd set ao/aoh
        P.multiset = 1
        P.ae = _triple([float(x) for x in spec.get("ae", a)])
        P.aeh = _triple([float(x) for x in spec.get("aeh", ah)])
        P.ao = _triple([float(x) for x in spec.get("ao", a)])
        P.aoh = _triple([float(x) for x in spec.get("aoh", ah)])
    return P


def _with_boundary(P, bc):
    """Dirichlet edges: bc = dict(G=values per node, scale=exp(lambda t) of
    the level written).  The array is kept alive on the parameter block."""
    if bc is None:
        return P
    G = np.ascontiguousarray(bc["G"], dtype=np.float64).ravel()
    P.bc = 1
    P.bscale = float(bc["scale"])
    P.bG = G.ctypes.data_as(C.POINTER(C.c_double))
    P._keep = G
    return P


def nfields(spec) -> int:
    return 1 + DIMS[spec["lattice"]] if spec.get("eq", "lcde") == "nse" else 1


def npoints(spec) -> int:
    return int(np.prod(spec["n"]))


def _check(rc, name):
    if rc < 0:
        raise RuntimeError("%s failed (%d)" % (name, rc))


def make_source(src: dict) -> Source:
    """src keys: b, bh (k = -1, 0, 1 at levels t and t - dt), v (M_1F = v S)."""
    Q = Source()
    Q.b = _triple([float(x) for x in src.get("b", (0.0, 0.0, 0.0))])
    Q.bh = _triple([float(x) for x in src.get("bh", (0.0, 0.0, 0.0))])
    Q.v = _triple([float(x) for x in src.get("v", ())])
    return Q


def _source_step(fn, name, spec, cur, prev, src):
    P = make_params(spec)
    Q = make_source(src)
    out = np.empty_like(cur)
    prev = cur if prev is None else prev
    St = np.ascontiguousarray(src["S_t"], dtype=np.float64)
    Sm = np.ascontiguousarray(src["S_m"], dtype=np.float64)
    assert St.size == cur.size and Sm.size == cur.size
    _check(fn(C.byref(P), C.byref(Q), _ptr(cur), _ptr(prev), _ptr(St), _ptr(Sm), _ptr(out)), name)
    return out


def mmfd_step(spec, cur, prev=None, src=None, bc=None):
    """One MMFD step; src (linear CDE only): dict(b, bh, v, S_t, S_m) adds the
    scheme's source term with S given at levels t and t - dt; bc (2D scalar
    equations): dict(G, scale) sets the edge nodes of the new level to
    G * scale (Dirichlet)."""
    if src is not None:
        return _source_step(lib().orc_mmfd_source_step, "mmfd_source_step", spec, cur, prev, src)
    P = _with_boundary(make_params(spec), bc)
    out = np.empty_like(cur)
    prev = cur if prev is None else prev
    _check(lib().orc_mmfd_step(C.byref(P), _ptr(cur), _ptr(prev), _ptr(out)), "mmfd_step")
    return out


def literal_step(spec, cur, prev=None, src=None, bc=None):
    if src is not None:
        return _source_step(lib().orc_literal_source_step, "literal_source_step", spec, cur, prev,
                            src)
    P = _with_boundary(make_params(spec), bc)
    out = np.empty_like(cur)
    prev = cur if prev is None else prev
    _check(lib().orc_literal_step(C.byref(P), _ptr(cur), _ptr(prev), _ptr(out)), "literal_step")
    return out


def wave_start(spec, phi0, phit, bc=None):
    """Special first step of the three-level wave scheme (orc_wave_start)."""
    P = _with_boundary(make_params(spec), bc)
    out = np.empty_like(phi0)
    phit = np.ascontiguousarray(phit, dtype=np.float64)
    _check(lib().orc_wave_start(C.byref(P), _ptr(phi0), _ptr(phit), _ptr(out)), "wave_start")
    return out


def init_populations(spec, mom):
    P = make_params(spec)
    pop = np.empty((QS[spec["lattice"]] * npoints(spec),))
    _check(lib().orc_init_populations(C.byref(P), _ptr(mom), _ptr(pop)), "init_populations")
    return pop


def moments(spec, pop):
    P = make_params(spec)
    mom = np.empty((nfields(spec) * npoints(spec),))
    _check(lib().orc_moments(C.byref(P), _ptr(pop), _ptr(mom)), "moments")
    return mom


def mesofd_step(spec, pop, prev_mom=None, src=None):
    """Returns (new populations, moments of the input level); src (linear
    CDE): dict(b, bh, v, S_t, S_m) adds each direction's source term."""
    P = make_params(spec)
    out = np.empty_like(pop)
    mom_out = np.empty((nfields(spec) * npoints(spec),))
    if prev_mom is None:
        prev_mom = np.zeros_like(mom_out)  # read only by three-level schemes
    if src is not None:
        Q = make_source(src)
        St = np.ascontiguousarray(src["S_t"], dtype=np.float64)
        Sm = np.ascontiguousarray(src["S_m"], dtype=np.float64)
        assert St.size == npoints(spec) and Sm.size == npoints(spec)
        _check(lib().orc_mesofd_source_step(C.byref(P), C.byref(Q), _ptr(pop), _ptr(prev_mom),
                                            _ptr(St), _ptr(Sm), _ptr(out), _ptr(mom_out)),
               "mesofd_source_step")
        return out, mom_out
    _check(lib().orc_mesofd_step(C.byref(P), _ptr(pop), _ptr(prev_mom), _ptr(out), _ptr(mom_out)),
           "mesofd_step")
    return out, mom_out


def theta_step(spec, cur):
    P = make_params(spec)
    out = np.empty_like(cur)
    work = np.empty_like(cur)
    _check(lib().orc_theta_step(C.byref(P), _ptr(cur), _ptr(out), _ptr(work)), "theta_step")
    return out


def theta_solve(spec, cur, tol, chunk, cap):
    """Theta step solved to a tolerance (orc_theta_solve): returns
    (phi(t + dt), sweeps, converged)."""
    P = make_params(spec)
    out = np.empty_like(cur)
    work = np.empty_like(cur)
    sw, cv = C.c_int(), C.c_int()
    _check(lib().orc_theta_solve(C.byref(P), _ptr(cur), _ptr(out), _ptr(work), float(tol),
                                 int(chunk), int(cap), C.byref(sw), C.byref(cv)), "theta_solve")
    return out, sw.value, bool(cv.value)


def pair_parts(spec, lev):
    """(Fp[p, N], Fm[p, N]): the pair parts of one level as the central form
    uses them (orc_pair_parts)."""
    P = make_params(spec)
    lev = np.ascontiguousarray(lev, dtype=np.float64)
    N = npoints(spec)
    Fp = np.zeros(MAXP * N)
    Fm = np.zeros(MAXP * N)
    npair = lib().orc_pair_parts(C.byref(P), _ptr(lev), _ptr(Fp), _ptr(Fm))
    _check(npair, "pair_parts")
    return Fp[: npair * N].reshape(npair, N), Fm[: npair * N].reshape(npair, N)


def tables(spec):
    """(w[b], ubar[b], dict of per-pair ubp, ubm, Cp, Cm, Chp, Chm)."""
    P = make_params(spec)
    b = QS[spec["lattice"]]
    w = np.zeros(b)
    ub = np.zeros(b)
    p6 = np.zeros(6 * MAXP)
    _check(lib().orc_tables(C.byref(P), _ptr(w), _ptr(ub), _ptr(p6)), "tables")
    npair = (b - 1) // 2
    p6 = p6.reshape(6, MAXP)[:, :npair]
    names = ["ubp", "ubm", "Cp", "Cm", "Chp", "Chm"]
    return w, ub, {k: p6[i].copy() for i, k in enumerate(names)}


def lattice_info(lattice, d0=1.0 / 3.0):
    """(e[b,3] int, w[b], pair representatives)."""
    e = (C.c_int * (3 * MAXQ))()
    w = np.zeros(MAXQ)
    npair = C.c_int()
    pairs = (C.c_int * MAXP)()
    b = lib().orc_lattice_info(LATTICES[lattice], d0, e, _ptr(w), C.byref(npair), pairs)
    _check(b, "lattice_info")
    E = np.array(e[: 3 * b], dtype=np.int64).reshape(b, 3)
    return E, w[:b].copy(), [pairs[i] for i in range(npair.value)]


def edf(lattice, d0, A, B, Cm):
    """g_j(A, B, C) of Eq. (3-3) in lattice units, all j."""
    B3 = np.zeros(3)
    B3[: len(B)] = B
    C9 = np.zeros((3, 3))
    Cm = np.asarray(Cm, dtype=np.float64)
    C9[: Cm.shape[0], : Cm.shape[1]] = Cm
    C9 = np.ascontiguousarray(C9.ravel())
    g = np.zeros(MAXQ)
    b = lib().orc_edf(LATTICES[lattice], d0, float(A), _ptr(np.ascontiguousarray(B3)), _ptr(C9), _ptr(g))
    _check(b, "edf")
    return g[:b].copy()


def lattice_info_rect(lattice, d0v):
    """(e[b,3] int, w[b], pair representatives) with d0 per axis."""
    e = (C.c_int * (3 * MAXQ))()
    w = np.zeros(MAXQ)
    npair = C.c_int()
    pairs = (C.c_int * MAXP)()
    dv = np.ascontiguousarray((list(d0v) + [d0v[0]] * 3)[:3], dtype=np.float64)
    b = lib().orc_lattice_info_rect(LATTICES[lattice], _ptr(dv), e, _ptr(w), C.byref(npair), pairs)
    _check(b, "lattice_info_rect")
    E = np.array(e[: 3 * b], dtype=np.int64).reshape(b, 3)
    return E, w[:b].copy(), [pairs[i] for i in range(npair.value)]


def edf_rect(lattice, d0v, A, B, Cm):
    """g_j(A, B, C) of Eq. (3-3) in lattice units with d0 per axis, all j."""
    B3 = np.zeros(3)
    B3[: len(B)] = B
    C9 = np.zeros((3, 3))
    Cm = np.asarray(Cm, dtype=np.float64)
    C9[: Cm.shape[0], : Cm.shape[1]] = Cm
    C9 = np.ascontiguousarray(C9.ravel())
    dv = np.ascontiguousarray((list(d0v) + [d0v[0]] * 3)[:3], dtype=np.float64)
    g = np.zeros(MAXQ)
    b = lib().orc_edf_rect(LATTICES[lattice], _ptr(dv), float(A), _ptr(np.ascontiguousarray(B3)),
                           _ptr(C9), _ptr(g))
    _check(b, "edf_rect")
    return g[:b].copy()


def csum(v) -> float:
    """Neumaier-compensated FP64 sum."""
    v = np.ascontiguousarray(v, dtype=np.float64).ravel()
    return lib().orc_sum(_ptr(v), v.size)
