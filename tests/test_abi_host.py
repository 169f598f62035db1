"""CPU checks of the C ABI: every symbol include/mfd.h declares is exported by
libmfd.so, argument validation, and the host-side algebra (coefficient
moments, Eq. (X), presets, transport coefficients, the per-pair EDF
constants) against the oracle's independent implementation -- no GPU work."""
import ctypes as C
import os
import re
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import native as O
from oracle import scheme as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "mfd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mfd_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported(M):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(M.lib, n), n


def test_coeff_moments_match_oracle(M):
    rng = np.random.default_rng(0)
    for _ in range(30):
        a = [float(F(int(v), 8)) for v in rng.integers(-16, 17, 3)]
        ah = [float(F(int(v), 8)) for v in rng.integers(-16, 17, 3)]
        m = S.coeff_moments(a, ah)
        got = M.mfd_coeff_moments(a, ah)
        want = [m[(0, 0)], m[(1, 0)], m[(1, 1)], m[(2, 0)], m[(2, 1)], m[(2, 2)]]
        assert got == [float(x) for x in want]


def test_constraint_solve_matches_oracle(M):
    rng = np.random.default_rng(1)
    for _ in range(30):
        g = [F(int(v), 8) for v in rng.integers(-16, 17, 5)]
        a, ah = S.solve_constraints(*g)
        ga, gah = M.mfd_coeffs_from_constraints(*[float(x) for x in g])
        assert list(ga) == [float(x) for x in a] and list(gah) == [float(x) for x in ah]


@pytest.mark.parametrize("name,param", [("srt", 0.0), ("trt", 0.625), ("one_stage", 1.25),
                                        ("two_level", 0.75)])
def test_presets_match_oracle(M, name, param):
    fn = {"srt": lambda p: S.preset_srt(), "trt": S.preset_trt, "one_stage": S.preset_one_stage,
          "two_level": S.preset_two_level}[name]
    a, ah = fn(F(param))
    ga, gah = M.mfd_preset(name, param)
    assert list(ga) == [float(x) for x in a] and list(gah) == [float(x) for x in ah]


def test_transport_coefficient(M):
    s = F(2, 3)
    a, ah = S.preset_trt(s)
    nu = S.viscosity(a, ah, F(1, 64), F(1, 4096), F(1, 3))
    got = M.mfd_transport_coefficient([float(x) for x in a], [float(x) for x in ah],
                                      1 / 64, 1 / 4096, 1 / 3)
    assert abs(got - float(nu)) <= 1e-15 * float(nu)


LIN = [
    ("D1Q3", dict(n=(16,), u=(0.3,), K=[[0.4]]), (1.25, -0.5, 0.25), None),
    ("D2Q9", dict(n=(16, 16), u=(0.05, 0.03), K=[[0.02, 0.005], [0.005, 0.01]], dx=1 / 2048,
                  dt=2.0 ** -18, lambda_bar=1), (1.0, 0.0, 0.0), None),
    ("D2Q9", dict(n=(8, 8), u=(0.3, -0.2), K=[[0.3, 0.05], [0.05, 0.2]], lambda_bar=1),
     (0.875, 0.0, 0.125), (0.125, 0.0, -0.125)),
    ("D3Q19", dict(n=(5, 5, 5), u=(0.1, 0.2, -0.1), K=[[0.2, 0.01, 0.0], [0.01, 0.3, 0.02], [0.0, 0.02, 0.25]],
                   lambda_bar=1), (1.0, 0.0, 0.4), (0.0, -0.4, 0.0)),
    ("D2Q5II", dict(n=(8, 6), u=(0.1, -0.2), K=[[0.2, 0.0], [0.0, 0.2]], d0=0.4), (1.0, 0.0, 0.0), None),
    ("D3Q7", dict(n=(4, 5, 6), u=(0.1, 0.2, -0.1), K=[[0.15, 0.0, 0.0], [0.0, 0.15, 0.0], [0.0, 0.0, 0.15]],
                  d0=0.25), (1.0, 0.0, 0.4), (0.0, -0.4, 0.0)),
    ("D3Q9", dict(n=(4, 5, 6), u=(0.1, 0.2, -0.1), K=[[0.2, 0.0, 0.0], [0.0, 0.2, 0.0], [0.0, 0.0, 0.2]]),
     (1.1, -0.2, 0.1), None),
    # rectangular lattices: spacing and d0 per axis
    ("D2Q9", dict(n=(8, 6), u=(0.3, -0.2), K=[[0.3, 0.05], [0.05, 0.2]], lambda_bar=1,
                  dxv=(0.5, 2.0), d0v=(0.3, 0.45), dt=0.1), (1.0, 0.0, 0.0), None),
    ("D2Q5", dict(n=(8, 6), u=(0.3, -0.2), K=[[0.3, 0.0], [0.0, 0.2]], dxv=(1.0, 1.5),
                  d0v=(0.3, 0.2), dt=0.2), (0.875, 0.0, 0.125), (0.125, 0.0, -0.125)),
    ("D3Q19", dict(n=(4, 5, 6), u=(0.1, 0.2, -0.1), K=[[0.2, 0.01, 0.0], [0.01, 0.3, 0.02], [0.0, 0.02, 0.25]],
                   lambda_bar=1, dxv=(1.0, 0.5, 2.0), d0v=(0.3, 0.25, 0.2), dt=0.05), (1.0, 0.0, 0.4),
     (0.0, -0.4, 0.0)),
    ("D3Q7", dict(n=(4, 5, 6), u=(0.1, 0.2, -0.1), K=[[0.15, 0.0, 0.0], [0.0, 0.25, 0.0], [0.0, 0.0, 0.1]],
                  dxv=(1.0, 1.25, 0.75), d0v=(0.3, 0.2, 0.25), dt=0.1), (1.0, 0.0, 0.0), None),
]


@pytest.mark.parametrize("lat,kw,a,ah", LIN, ids=["d1q3", "d2q9-c2", "d2q9-3l", "d3q19-trt", "d2q5ii",
                                                   "d3q7-trt", "d3q9", "rect-d2q9", "rect-d2q5-3l",
                                                   "rect-d3q19-trt", "rect-d3q7"])
def test_linear_constant_tables_bitwise(M, lat, kw, a, ah):
    """The library's and the oracle's EDF constants are formed independently
    from the same formulas; FP64 parity requires them to be identical."""
    kind = "three_level" if ah else "two_level"
    spec = dict(lattice=lat, eq="lcde", a=a, ah=ah or (0, 0, 0), levels=3 if ah else 2,
                dx=kw.get("dx", 1.0), dt=kw.get("dt", 1.0), **{k: v for k, v in kw.items() if k not in ("dx", "dt")})
    w, ub, tab = O.tables(spec)
    s = M.Solver(lat, kw["n"], kw.get("dx", 1.0), "fp64", "mmfd", d0=kw.get("d0", 1.0 / 3.0))
    if "dxv" in kw:
        s.set_rectangular(kw["dxv"], kw["d0v"])
    s.set_equation("lcde", u=kw["u"], K=kw["K"], lambda_bar=kw.get("lambda_bar", 0))
    s.set_scheme(kind, a, ah, dt=kw.get("dt", 1.0))
    gw, gub, gtab = s.linear_tables()
    assert np.array_equal(gw, w) and np.array_equal(gub, ub)
    for k in tab:
        assert np.array_equal(gtab[k], tab[k]), k
    s.close()


def test_max_amplification_matches_oracle(M):
    kw = dict(n=(12, 10), u=(0.9, 0.7), K=[[0.02, 0.0], [0.0, 0.02]], lambda_bar=1)
    a, ah = (1.0, 0.0, 0.0), (0.5, -1.0, 0.5)
    spec = dict(lattice="D2Q9", eq="lcde", a=a, ah=ah, levels=3, **kw)
    E, w, pairs = O.lattice_info("D2Q9")
    _, _, tab = O.tables(spec)
    want = S.max_amplification(E, pairs, tab["ubp"], tab["ubm"], kw["n"], a, ah)
    s = M.Solver("D2Q9", kw["n"], 1.0, "fp64", "mmfd")
    s.set_equation("lcde", u=kw["u"], K=kw["K"], lambda_bar=1)
    s.set_scheme("three_level", a, ah, dt=1.0)
    assert abs(s.max_amplification() - want) < 1e-12
    s.close()


def test_argument_validation(M):
    with pytest.raises(M.MfdError):
        M.Solver("D2Q9", (2, 8), 1.0)  # fewer than 3 nodes
    with pytest.raises(M.MfdError):
        M.Solver("D2Q9", (8, 8), -1.0)  # dx <= 0
    s = M.Solver("D2Q9", (8, 8), 1.0)
    with pytest.raises(M.MfdError) as e:
        s.set_scheme("two_level", (1, 0, 0), dt=1.0)  # equation not set
    assert e.value.code == M.MFD_E_ORDER
    with pytest.raises(M.MfdError) as e:
        s.set_lattice("D3Q19")  # dimension mismatch
    assert e.value.code == M.MFD_E_ARG
    s.set_equation("burgers", beta=0.5)
    with pytest.raises(M.MfdError) as e:  # theta: LCDE, Burgers at beta = 1 and the NSE
        s.set_scheme("theta", (1, 0, 0), theta=0.5, theta_iters=3, dt=1.0)
    assert e.value.code == M.MFD_E_UNSUPPORTED
    s.set_equation("nse", rho0=1.0)
    s.set_scheme("theta", (1, 0, 0), theta=0.5, theta_iters=3, dt=1.0)
    with pytest.raises(M.MfdError) as e:
        s.step(1)  # no state
    assert e.value.code == M.MFD_E_ORDER
    # inconsistent coefficients are a warning, not an error
    rc = s.set_scheme("two_level", (1.0, 0.5, 0.0), dt=1.0)
    assert rc == M.MFD_W_INCONSISTENT
    s.close()
    s = M.Solver("D1Q3", (8,), 1.0)
    with pytest.raises(M.MfdError) as e:
        s.set_equation("nse", rho0=1.0)
    assert e.value.code == M.MFD_E_UNSUPPORTED
    s.close()


def test_source_argument_validation(M):
    """mfd_set_source checks order, form, equation, scheme kind, count and
    finiteness before it touches the device."""
    G = np.zeros(64)
    s = M.Solver("D2Q9", (8, 8), 1.0)
    with pytest.raises(M.MfdError) as e:
        s.set_source(G)  # not configured
    assert e.value.code == M.MFD_E_ORDER
    s.set_equation("lcde", u=(0.01, 0.0), K=[[0.1, 0.0], [0.0, 0.1]])
    s.set_scheme("two_level", (1, 0, 0), dt=1.0)
    with pytest.raises(M.MfdError) as e:
        s.set_source(G[:-1])
    assert e.value.code == M.MFD_E_ARG
    bad = G.copy()
    bad[3] = np.inf
    with pytest.raises(M.MfdError) as e:
        s.set_source(bad)
    assert e.value.code == M.MFD_E_ARG
    with pytest.raises(M.MfdError) as e:
        s.set_source(G, lam=float("nan"))
    assert e.value.code == M.MFD_E_ARG
    s.close()
    for form, eq, kind in (("mmfd", "burgers", "two_level"), ("mmfd", "lcde", "theta")):
        s = M.Solver("D2Q9", (8, 8), 1.0, "fp64", form)
        s.set_equation(eq, u=(0.01, 0.0), K=[[0.1, 0.0], [0.0, 0.1]])
        s.set_scheme(kind, (1, 0, 0), theta=0.5, theta_iters=2, dt=1.0)
        with pytest.raises(M.MfdError) as e:
            s.set_source(G)
        assert e.value.code == M.MFD_E_UNSUPPORTED
        s.close()
    s = M.Solver("D3Q19", (4, 4, 4), 1.0, "fp64", "mesofd")  # MesoFD with a source: 1D / 2D
    s.set_equation("lcde", u=(0.01, 0.0, 0.0), K=np.eye(3).tolist())
    s.set_scheme("two_level", (1, 0, 0), dt=1.0)
    with pytest.raises(M.MfdError) as e:
        s.set_source(np.zeros(64))
    assert e.value.code == M.MFD_E_UNSUPPORTED
    s.close()


def test_stability_warning(M):
    """Theorem 1 for C1-like D1Q3 schemes: r = 0.25 proven, r = 0.55 not."""
    for r, want in ((0.25, 0), (0.55, M.MFD_W_STABILITY_UNPROVEN)):
        s = M.Solver("D1Q3", (16,), 1.0)
        s.set_equation("lcde", u=(0.01,), K=[[1.0]])
        sp = 2 * r / (1 / 3)
        a, _ = M.mfd_preset("two_level", sp)
        assert s.set_scheme("two_level", a, dt=r) == want
        s.close()


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The binding has no fallback: loaded from a directory without
    libmfd.so it raises at import."""
    import importlib.util
    import shutil
    src = os.path.join(os.path.dirname(__file__), "..", "paper_2505_17057_amd", "mfd.py")
    dst = tmp_path / "mfd_copy.py"
    shutil.copy(src, dst)
    spec = importlib.util.spec_from_file_location("mfd_copy", dst)
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError, match="libmfd.so is not built"):
        spec.loader.exec_module(mod)


@pytest.mark.parametrize("lat,n,u,alpha,dx", [
    ("D1Q3", (1024,), (0.1,), 0.01, 1.0 / 1024),
    ("D1Q3", (64,), (2.0,), 0.05, 1.0 / 64),
    ("D2Q9", (24, 20), (0.9, 0.7), 0.02, 0.05),
    ("D2Q5", (16, 18), (0.3, -0.2), 0.01, 0.1),
    ("D3Q19", (6, 5, 4), (0.2, 0.1, -0.3), 0.01, 0.1),
])
def test_max_stable_dt_matches_oracle(M, lat, n, u, alpha, dx):
    """mfd_max_stable_dt: the sufficient bound equals Eq. (LMMFD-2-3) of the
    oracle's algebra; the exact bound sits where the oracle's Fourier symbol
    of the m = 1 two-level family (Eq. (LMMFD-2-2) coefficients, linear EDF)
    crosses |lambda| = 1 on the same periodic grid."""
    _, w, pairs = O.lattice_info(lat)
    E, _, _ = O.lattice_info(lat)
    d0 = 1.0 / 3.0
    suff, exact = M.mfd_max_stable_dt(lat, dx, u, alpha, n=n)
    want = S.linear_edf_bound_dt(alpha, np.array(u, dtype=float), dx, (d0, w[0]))
    assert suff == pytest.approx(want, rel=1e-15)
    assert exact >= suff * (1 - 1e-12)  # Eq. (LMMFD-2-3) is sufficient

    def amp(dt):
        s = 2 * alpha * dt / (d0 * dx * dx)
        a = ((s + 1) / 2, 1 - s, (s - 1) / 2)  # a_{-1}, a_0, a_1
        uh = np.array(list(u) + [0.0] * (3 - len(u))) * dt / dx
        ubp = [w[j] for j in pairs]
        ubm = [w[j] * float(np.dot(E[j], uh)) / d0 for j in pairs]
        return S.max_amplification(E, pairs, ubp, ubm, n, a, (0.0, 0.0, 0.0))

    assert amp(exact * (1 - 1e-9)) <= 1 + 1e-12
    assert amp(exact * (1 + 1e-6)) > 1 + 1e-13
    assert amp(suff) <= 1 + 1e-12


def test_c1_time_step_is_half_the_library_bound(M):
    """The 1D workload's dt = 25 * 2^-20 is half the Eq. (LMMFD-2-3) bound the
    library reports for D1Q3, N = 1024, u = 0.1, D = 0.01."""
    from mfd_inputs import c1_linear_1d

    c1 = c1_linear_1d()
    suff, _ = M.mfd_max_stable_dt("D1Q3", c1["dx"], c1["u"], c1["D"])
    assert 0.5 * suff == pytest.approx(c1["dt"], rel=1e-14)


def test_max_stable_dt_argument_checks(M):
    import ctypes as C

    d = C.c_double()
    u = (C.c_double * 3)(0.1, 0.0, 0.0)
    assert M.lib.mfd_max_stable_dt(1, 0.0, 0.0, u, 0.01, None, C.byref(d), None) == M.MFD_E_ARG
    assert M.lib.mfd_max_stable_dt(1, 0.0, 0.1, u, -1.0, None, C.byref(d), None) == M.MFD_E_ARG
    assert M.lib.mfd_max_stable_dt(9, 0.0, 0.1, u, 0.01, None, C.byref(d), None) == M.MFD_E_ARG
    assert M.lib.mfd_max_stable_dt(1, 0.0, 0.1, None, 0.01, None, C.byref(d), None) == M.MFD_E_ARG
    big = (C.c_int64 * 3)(1 << 13, 1 << 13, 1)
    e = C.c_double()
    assert M.lib.mfd_max_stable_dt(3, 0.0, 0.1, u, 0.01, big, C.byref(d), C.byref(e)) == M.MFD_E_ARG



@pytest.mark.parametrize("lat,beta,gamma", [("D2Q5", 1.0, 0.375), ("D2Q9", 1.0, 0.375),
                                            ("D2Q9", 0.75, 0.5), ("D3Q19", 1.25, 0.3)])
def test_wave_constant_tables_bitwise(M, lat, beta, gamma):
    """The wave EDF table (Example 3) of the library equals the oracle's bit
    for bit, and the configured three-level wave scheme is neutral (largest
    root modulus 1) on a periodic grid."""
    n = (9,) * O.DIMS[lat]
    a, ah = (gamma, 2 * (1 - gamma), gamma), (0.0, -1.0, 0.0)
    spec = dict(lattice=lat, eq="wave", n=n, beta=beta, a=a, ah=ah, levels=3)
    w, ub, tab = O.tables(spec)
    s = M.Solver(lat, n, 1.0, "fp64", "mmfd")
    s.set_equation("wave", beta=beta)
    s.set_scheme("three_level", a, ah, dt=1.0)
    gw, gub, gtab = s.linear_tables()
    assert np.array_equal(gw, w) and np.array_equal(gub, ub)
    for k in tab:
        assert np.array_equal(gtab[k], tab[k]), k
    assert abs(s.max_amplification() - 1.0) < 1e-12
    s.close()


def test_dirichlet_argument_checks(M):
    """Dirichlet grids are 2D MMFD; scalar equations only; periodic grids have
    no boundary values; the first wave step needs a three-level wave scheme."""
    with pytest.raises(M.MfdError) as ei:
        M.Solver("D1Q3", (16,), 1.0, "fp64", "mmfd", boundary="dirichlet")
    assert ei.value.code == M.MFD_E_UNSUPPORTED
    with pytest.raises(M.MfdError) as ei:
        M.Solver("D2Q9", (16, 16), 1.0, "fp64", "mesofd", boundary="dirichlet")
    assert ei.value.code == M.MFD_E_UNSUPPORTED
    s = M.Solver("D2Q9", (16, 16), 1.0, "fp64", "mmfd", boundary="dirichlet")
    with pytest.raises(M.MfdError) as ei:
        s.set_equation("nse", rho0=1.0)
    assert ei.value.code == M.MFD_E_UNSUPPORTED
    s.set_equation("lcde", u=(0.1, 0.0), K=[[0.1, 0], [0, 0.1]])
    with pytest.raises(M.MfdError) as ei:
        s.set_scheme("theta", (1.0, 0.0, 0.0), theta=0.5, theta_iters=4)
    assert ei.value.code == M.MFD_E_UNSUPPORTED
    with pytest.raises(M.MfdError):
        s.set_boundary(np.zeros(10))  # wrong count
    with pytest.raises(M.MfdError):
        s.set_boundary(np.full(256, np.nan))
    s.close()
    p = M.Solver("D2Q9", (16, 16), 1.0, "fp64", "mmfd")
    p.set_equation("wave", beta=1.0)
    p.set_scheme("three_level", (0.375, 1.25, 0.375), (0.0, -1.0, 0.0), dt=1.0)
    with pytest.raises(M.MfdError) as ei:
        p.set_boundary(np.zeros(256))
    assert ei.value.code == M.MFD_E_ORDER
    with pytest.raises(M.MfdError) as ei:
        p.wave_start(np.zeros(256))  # no state yet
    assert ei.value.code == M.MFD_E_ORDER
    p.close()


@pytest.mark.parametrize("three", [False, True])
def test_multiset_constant_tables_bitwise(M, three):
    """The multiple-set constants (Eq. (2-2-1b)) of the library equal the
    oracle's bit for bit."""
    kw = dict(n=(8, 8), u=(0.3, -0.2), K=[[0.3, 0.05], [0.05, 0.2]], lambda_bar=1)
    a, ah = ((0.875, 0.0, 0.125), (0.125, 0.0, -0.125)) if three else ((0.6, 0.2, 0.2), None)
    ae, aeh = (0.8, 0.1, 0.1), (0.1, -0.1, 0.1)
    ao, aoh = (0.95, 0.0, 0.05), (0.05, 0.0, -0.05)
    spec = dict(lattice="D2Q9", eq="lcde", a=a, ae=ae, ao=ao, levels=3 if three else 2, **kw)
    if three:
        spec.update(ah=ah, aeh=aeh, aoh=aoh)
    w, ub, tab = O.tables(spec)
    s = M.Solver("D2Q9", kw["n"], 1.0, "fp64", "mmfd")
    s.set_equation("lcde", u=kw["u"], K=kw["K"], lambda_bar=1)
    if three:
        s.set_scheme_sets("three_level", a, ae, ao, ah, aeh, aoh, dt=1.0)
    else:
        s.set_scheme_sets("two_level", a, ae, ao, dt=1.0)
    gw, gub, gtab = s.linear_tables()
    assert np.array_equal(gub, ub)
    for k in tab:
        assert np.array_equal(gtab[k], tab[k]), k
    s.close()


def test_theta_multigrid_argument_checks(M):
    """mfd_set_theta_multigrid: theta scheme first; the 2D linear CDE on
    D2Q5 / D2Q9 only; levels the grid allows (halving while both sides stay
    even and >= 4); pre in [1, 8], post in [0, 8]; 0 switches it off."""
    s = M.Solver("D2Q9", (96, 64), 1.0, "fp64", "mmfd")
    s.set_equation("lcde", u=(0.1, 0.0), K=[[1.0, 0], [0, 1.0]])
    s.set_scheme("two_level", (1.0, 0.0, 0.0), dt=1.0)
    with pytest.raises(M.MfdError) as ei:
        s.set_theta_multigrid(-1)
    assert ei.value.code == M.MFD_E_ORDER
    s.set_scheme("theta", (1.0, 0.0, 0.0), theta=0.5, theta_iters=20)
    s.set_theta_multigrid(-1)          # (96,64) (48,32) (24,16) (12,8) (6,4): 5 levels
    s.set_theta_multigrid(5, 1, 0)
    for bad in ((6, 2, 2), (1, 2, 2), (3, 0, 2), (3, 9, 2), (3, 2, 9), (3, 2, -1)):
        with pytest.raises(M.MfdError) as ei:
            s.set_theta_multigrid(*bad)
        assert ei.value.code == M.MFD_E_ARG, bad
    s.set_theta_multigrid(0)
    s.close()
    s = M.Solver("D2Q9", (32, 32), 1.0, "fp64", "mmfd")
    s.set_equation("burgers", beta=1.0)
    s.set_scheme("theta", (1.0, 0.0, 0.0), theta=0.5, theta_iters=20)
    with pytest.raises(M.MfdError) as ei:
        s.set_theta_multigrid(-1)
    assert ei.value.code == M.MFD_E_UNSUPPORTED
    s.set_theta_multigrid(0)  # off is always accepted
    s.close()
    s = M.Solver("D1Q3", (64,), 1.0, "fp64", "mmfd")
    s.set_equation("lcde", u=(0.1,), K=[[1.0]])
    s.set_scheme("theta", (1.0, 0.0, 0.0), theta=0.5, theta_iters=20)
    with pytest.raises(M.MfdError) as ei:
        s.set_theta_multigrid(-1)
    assert ei.value.code == M.MFD_E_UNSUPPORTED
    s.close()


def test_rectangular_argument_checks(M):
    """mfd_set_rectangular: after the lattice; the linear CDE only (either
    order); one d0 on rD2Q5II / rD3Q9; d0 in (0, 1), positive spacing and
    weights; no source term; a new lattice returns to the square one."""
    s = M.Solver("D2Q9", (8, 8), 1.0, "fp64", "mmfd")
    s.set_rectangular((0.5, 2.0), (0.3, 0.4))
    with pytest.raises(M.MfdError) as e:
        s.set_equation("burgers", beta=1.0)
    assert e.value.code == M.MFD_E_UNSUPPORTED
    for bad in (((0.5, 2.0), (0.0, 0.4)), ((0.5, 2.0), (0.3, 1.0)), ((0.0, 2.0), (0.3, 0.4))):
        with pytest.raises(M.MfdError) as e:
            s.set_rectangular(*bad)
        assert e.value.code == M.MFD_E_ARG
    s.set_equation("lcde", u=(0.1, 0.0), K=[[0.1, 0], [0, 0.1]])
    s.set_scheme("two_level", (1.0, 0.0, 0.0), dt=0.1)
    with pytest.raises(M.MfdError) as e:
        s.set_source(np.zeros(64), 0.0, (0.0, 1.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0))
    assert e.value.code == M.MFD_E_UNSUPPORTED
    s.close()
    s = M.Solver("D2Q5", (8, 8), 1.0, "fp64", "mmfd")
    with pytest.raises(M.MfdError) as e:  # weight 1 - 0.6 - 0.5 < 0
        s.set_rectangular((1.0, 1.0), (0.6, 0.5))
    assert e.value.code == M.MFD_E_ARG
    s.close()
    s = M.Solver("D2Q5II", (8, 8), 1.0, "fp64", "mmfd")
    with pytest.raises(M.MfdError) as e:
        s.set_rectangular((1.0, 2.0), (0.3, 0.4))
    assert e.value.code == M.MFD_E_UNSUPPORTED
    s.set_rectangular((1.0, 2.0), (0.3, 0.3))  # one d0, two spacings
    s.close()
    s = M.Solver("D2Q9", (8, 8), 1.0, "fp64", "mmfd")
    s.set_equation("nse", rho0=1.0)
    with pytest.raises(M.MfdError) as e:
        s.set_rectangular((0.5, 2.0), (0.3, 0.4))
    assert e.value.code == M.MFD_E_UNSUPPORTED
    s.close()


def test_general_argument_checks(M):
    """mfd_general_create refuses bad sizes and coefficients before it
    allocates anything: m in [1, 3], n in [1, 4], finite coefficients with
    A10 < 0 < A22, a known precision, extents within the launch grid."""
    a1 = [[0.25, 0.5, 0.25, 0.0, 0.0]]
    bad = [
        dict(a=np.zeros((1, 9))),                      # m = 4
        dict(a=np.zeros((5, 3))),                      # n = 5
        dict(a=[[np.nan, 1.0, 0.0]]),
        dict(a=[[0.0, 1.0, 0.0]]),                     # A10 < 0 but A22 = 0
        dict(a=a1, dt=0.0),
        dict(a=a1, lattice="D2Q9", n=(8, 8), precision="fp16"),
        dict(a=a1, lattice="D2Q9", n=(1, 4 * 65535 + 1)),  # beyond the launch grid
        dict(a=a1, lattice="D3Q19", n=(1, 1, 65536), u=(0.1, 0.0, 0.0),
             K=np.eye(3).tolist()),
    ]
    for kw in bad:
        args = dict(lattice="D2Q9", n=(8, 8), dx=1.0, a=a1, dt=0.1, u=(0.1, 0.0),
                    K=[[0.1, 0.0], [0.0, 0.1]])
        args.update(kw)
        with pytest.raises((M.MfdError, KeyError)) as ei:
            M.General(**args)
        if ei.type is M.MfdError:
            assert ei.value.code == M.MFD_E_ARG, kw
