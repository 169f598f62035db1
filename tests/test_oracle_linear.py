"""Pins of the oracle's linear-CDE steps.

* Fourier symbol: one MMFD step multiplies each Fourier mode by A_{-1}(xi)
  (and adds A_{-2}(xi) times the older level for three-level schemes),
  Eq. (TforMMFD-3) -- an independent route through the mathematics that
  catches a wrong sign, index or transposed stencil.
* EDF constants: ubar_j satisfies the moment identities with the diffusion
  tensor recovered through alpha = -(A22/A10) dt beta c_s^2.
* FTCS: on D1Q3 the two-level m = 1 scheme is the textbook
  phi + r D2 phi - (C/2) D1 phi of Eq. (LMMFD-4a).
* LITERAL == MesoFD moments == MMFD up to round-off; conservation.
* theta scheme against its closed-form amplification, Eq. (Tcond1-1).
* stability: measured growth rate equals the exact max |lambda|.
"""
import numpy as np
import pytest

import mfd_inputs as I
from oracle import native as O
from oracle import scheme as S

LATS = ["D1Q3", "D2Q5", "D2Q9", "D3Q19", "D2Q5II", "D3Q7", "D3Q9"]
# lattices whose EDF meets the second-moment identity only for C = 0
C0_LATS = ("D2Q5", "D2Q5II", "D3Q7", "D3Q9")


def lin_spec(lat, case, a, ah=(0, 0, 0), lam=1, levels=None):
    dim = O.DIMS[lat]
    K = case["K"]
    if lat in C0_LATS:  # keep C = 0 there (see the EDF pins)
        lam = 0
    spec = dict(lattice=lat, n=case["n"], dx=case["dx"], dt=case["dt"], u=case["u"], K=K,
                lambda_bar=lam, a=a, ah=ah, levels=levels or (3 if any(ah) else 2))
    if lat in C0_LATS:
        m = S.coeff_moments(a, ah)
        ratio = -m[(1, 0)] / m[(2, 2)]
        # isotropic K that makes C = ratio*kh - d0 I vanish
        spec["K"] = (np.eye(dim) * (1.0 / 3.0) / ratio).tolist()
    return spec


def fourier_residual(spec, cur, prev):
    out = O.mmfd_step(spec, cur, prev)
    E, w, pairs = O.lattice_info(spec["lattice"], spec.get("d0", 1 / 3))
    _, _, tab = O.tables(spec)
    n = spec["n"]
    shape = tuple(reversed(n))
    A1, A2 = S.fourier_symbols(E, pairs, tab["ubp"], tab["ubm"], n, spec["a"], spec["ah"])
    fc = np.fft.fftn(cur.reshape(shape))
    fp = np.fft.fftn(prev.reshape(shape))
    fo = np.fft.fftn(out.reshape(shape))
    pred = A1 * fc + (A2 * fp if spec["levels"] == 3 else 0)
    return np.abs(fo - pred).max() / np.abs(fc).max()


SCHEMES = {
    "srt": ((1, 0, 0), (0, 0, 0)),
    "two_level_s": ((1.1, -0.2, 0.1), (0, 0, 0)),
    "trt": ((1, 0, 0.4), (0, -0.4, 0)),
    "ex1_case3": ((7 / 8, 0, 1 / 8), (1 / 8, 0, -1 / 8)),
    "ex2_case3": ((1, 0, 0), (0.5, -1, 0.5)),
}


@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("name", list(SCHEMES))
def test_fourier_symbol(lat, name):
    case = I.random_linear_case(O.DIMS[lat], seed=hash((lat, name)) % 1000)
    a, ah = SCHEMES[name]
    spec = lin_spec(lat, case, a, ah, levels=3 if any(ah) else 2)
    if spec["levels"] == 2:
        spec["ah"] = (0, 0, 0)
    res = fourier_residual(spec, case["phi0"], case["phim"])
    assert res < 1e-13


@pytest.mark.parametrize("lat", ["D1Q3", "D2Q9", "D3Q19"])
@pytest.mark.parametrize("lam", [0, 1])
def test_ubar_moments_recover_K(lat, lam):
    """sum ubar = 1, sum e ubar = uh, sum e e ubar = (-A10/A22) kh + lam uh uh."""
    dim = O.DIMS[lat]
    case = I.random_linear_case(dim, seed=3)
    for a, ah in SCHEMES.values():
        spec = lin_spec(lat, case, a, ah, lam=lam)
        _, ub, tab = O.tables(spec)
        E, _, pairs = O.lattice_info(lat)
        Ed = E[:, :dim]
        uh = np.array(case["u"]) * case["dt"] / case["dx"]
        kh = np.array(case["K"]) * case["dt"] / case["dx"] ** 2
        m = S.coeff_moments(a, ah)
        want2 = (-m[(1, 0)] / m[(2, 2)]) * kh + lam * np.outer(uh, uh)
        assert abs(ub.sum() - 1) < 1e-14
        assert np.allclose(Ed.T @ ub, uh, atol=1e-15)
        assert np.allclose(np.einsum("j,ja,jb->ab", ub, Ed, Ed), want2, atol=1e-14)
        # pair parts are the even / odd parts of ubar, Eq. (TforMMFD-2)
        for p, j in enumerate(pairs):
            jb = [i for i in range(len(ub)) if (E[i] == -E[j]).all()][0]
            assert abs(tab["ubp"][p] - 0.5 * (ub[j] + ub[jb])) < 1e-15
            assert abs(tab["ubm"][p] - 0.5 * (ub[j] - ub[jb])) < 1e-15


def test_c1_is_ftcs():
    """Eq. (LMMFD-4a): phi + r D2 phi - (C/2) D1 phi, r = D dt/dx^2, C = u dt/dx."""
    c1 = I.c1_linear_1d()
    s = 2 * c1["D"] * c1["dt"] / ((1 / 3) * c1["dx"] ** 2)
    spec = dict(lattice="D1Q3", n=c1["n"], dx=c1["dx"], dt=c1["dt"], u=c1["u"], K=c1["K"],
                lambda_bar=0, a=S.preset_two_level(s)[0])
    phi = c1["phi0"]
    out = O.mmfd_step(spec, phi)
    r = c1["D"] * c1["dt"] / c1["dx"] ** 2
    C = c1["u"][0] * c1["dt"] / c1["dx"]
    pp, pm = np.roll(phi, -1), np.roll(phi, 1)
    ftcs = phi + r * (pp - 2 * phi + pm) - 0.5 * C * (pp - pm)
    assert np.abs(out - ftcs).max() < 4 * np.finfo(float).eps * np.abs(phi).max()
    # the chosen dt is half the stability bound of Eq. (LMMFD-2-3): r = 1/4
    assert abs(r - 0.25) < 1e-15


@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("name", ["srt", "trt", "ex1_case3"])
def test_forms_agree_and_conserve(lat, name):
    case = I.random_linear_case(O.DIMS[lat], seed=21)
    a, ah = SCHEMES[name]
    spec = lin_spec(lat, case, a, ah)
    cur, prev = case["phi0"], case["phim"]
    mm = O.mmfd_step(spec, cur, prev)
    lit = O.literal_step(spec, cur, prev)
    pop = O.init_populations(spec, cur)
    newpop, mom_cur = O.mesofd_step(spec, pop, prev)
    meso = O.moments(spec, newpop)
    scale = np.abs(cur).max() + np.abs(prev).max()
    assert np.abs(mm - lit).max() < 1e-13 * scale
    assert np.abs(mm - meso).max() < 1e-13 * scale
    assert np.abs(mom_cur - cur).max() < 1e-14 * scale
    # conservation on a periodic grid: sum(out) = A0 sum(cur) + Ah0 sum(prev)
    want = sum(a) * O.csum(cur) + sum(ah) * O.csum(prev)
    assert abs(O.csum(mm) - want) < 1e-12 * np.abs(cur).sum()


@pytest.mark.parametrize("lat", ["D1Q3", "D2Q9", "D3Q19"])
@pytest.mark.parametrize("theta", [0.0, 0.5, 0.75])
def test_theta_closed_form(lat, theta):
    """Jacobi-solved theta step equals lambda = (1 + th z)/(1 - (1-th) z),
    z = A + iB of Eq. (Tcond1-2), mode by mode."""
    case = I.random_linear_case(O.DIMS[lat], seed=8)
    a = SCHEMES["two_level_s"][0]
    spec = lin_spec(lat, case, a)
    # keep the implicit operator diagonally dominant: scale the velocity down
    spec["u"] = tuple(0.3 * np.array(case["u"]))
    spec.update(theta=theta, theta_iters=200)
    cur = case["phi0"]
    out = O.theta_step(spec, cur)
    E, w, pairs = O.lattice_info(lat)
    _, _, tab = O.tables(spec)
    n = spec["n"]
    A1, _ = S.fourier_symbols(E, pairs, tab["ubp"], tab["ubm"], n, a, (0, 0, 0))
    z = A1 - 1.0
    lam = (1 + theta * z) / (1 - (1 - theta) * z)
    shape = tuple(reversed(n))
    fo = np.fft.fftn(out.reshape(shape))
    fc = np.fft.fftn(cur.reshape(shape))
    assert np.abs(fo - lam * fc).max() / np.abs(fc).max() < 1e-12


@pytest.mark.parametrize("lat", ["D2Q9", "D2Q5", "D1Q3"])
@pytest.mark.parametrize("tol,chunk", [(1e-6, 1), (1e-10, 3), (1e-12, 8)])
def test_theta_solve_to_tolerance(lat, tol, chunk):
    """The theta step solved to a residual tolerance (Eq. (GCN) with the
    stopping rule den ||x_k - x_(k-1)|| <= tol ||rhs||, checked every `chunk`
    sweeps):
    * the result lies within tol ||rhs|| of the exact theta solution, the
      closed form lambda = (A0 + th z)/(1 - (1-th) z) of Eq. (Tcond1-1) mode
      by mode (|1 - (1-th) z| >= 1 on a stable scheme, so the error is at most
      the residual of x_(k-1), which the rule bounds);
    * the sweep count is the first chunk boundary where the rule holds,
      recomputed here with numpy norms from fixed-count solves;
    * with the rule unreachable the solve stops at the cap and equals the
      fixed-count step."""
    case = I.random_linear_case(O.DIMS[lat], seed=9)
    a = SCHEMES["two_level_s"][0]
    theta = 0.5
    spec = lin_spec(lat, case, a)
    spec["u"] = tuple(0.3 * np.array(case["u"]))
    spec.update(theta=theta, theta_iters=1)
    cur = case["phi0"]
    out, sweeps, conv = O.theta_solve(spec, cur, tol, chunk, 400)
    assert conv and sweeps % chunk == 0
    E, w, pairs = O.lattice_info(lat)
    _, _, tab = O.tables(spec)
    n = spec["n"]
    A1, _ = S.fourier_symbols(E, pairs, tab["ubp"], tab["ubm"], n, a, (0, 0, 0))
    z = A1 - 1.0
    shape = tuple(reversed(n))
    fc = np.fft.fftn(cur.reshape(shape))
    exact = np.real(np.fft.ifftn((1 + theta * z) / (1 - (1 - theta) * z) * fc)).ravel()
    rhs = np.real(np.fft.ifftn((1 + theta * z) * fc)).ravel()
    err = np.linalg.norm(out - exact)
    assert err <= tol * np.linalg.norm(rhs) * 1.001 + 1e-13 * np.linalg.norm(exact)
    # the stopping point, from fixed-count solves and numpy norms
    den = 1.0 + (1 - theta) * 2 * float(np.sum(tab["ubp"]) * (a[0] + a[2]))

    def ratio(k):
        xk = O.theta_step(dict(spec, theta_iters=k), cur)
        xk1 = O.theta_step(dict(spec, theta_iters=k - 1), cur)
        return den * np.linalg.norm(xk - xk1) / np.linalg.norm(rhs)

    assert ratio(sweeps) <= tol * (1 + 1e-9)
    if sweeps > chunk:
        assert ratio(sweeps - chunk) > tol * (1 - 1e-9)
    fixed = O.theta_step(dict(spec, theta_iters=2 * chunk), cur)
    capped, k, c = O.theta_solve(spec, cur, 1e-300, chunk, 2 * chunk)
    assert k == 2 * chunk and not c and np.array_equal(capped, fixed)


def test_theta_one_is_explicit():
    case = I.random_linear_case(2, seed=4)
    spec = lin_spec("D2Q9", case, SCHEMES["two_level_s"][0])
    spec.update(theta=1.0, theta_iters=3)
    assert np.array_equal(O.theta_step(spec, case["phi0"]), O.mmfd_step(spec, case["phi0"]))


def test_stability_growth_matches_max_lambda():
    """C1 with r = D dt/dx^2 just above 1/2: lambda(pi) = 1 - 4r, so the
    highest mode grows by |1 - 4r| per step; just below 1/2 every mode except
    the conserved mean decays."""
    n = 16
    rng = np.random.default_rng(1)
    phi0 = rng.standard_normal(n)
    phi0 -= phi0.mean()
    for r, expect_growth in ((0.505, True), (0.49, False)):
        D, dx = 1.0, 1.0
        dt = r * dx * dx / D
        s = 2 * D * dt / ((1 / 3) * dx * dx)
        spec = dict(lattice="D1Q3", n=(n,), dx=dx, dt=dt, u=(0.0,), K=[[D]], a=S.preset_two_level(s)[0])
        E, w, pairs = O.lattice_info("D1Q3")
        _, _, tab = O.tables(spec)
        lam = S.max_amplification(E, pairs, tab["ubp"], tab["ubm"], (n,), spec["a"], (0, 0, 0))
        assert abs(lam - max(1.0, abs(1 - 4 * r))) < 1e-13
        phi = phi0.copy()
        norms = []
        for _ in range(400):
            phi = O.mmfd_step(spec, phi)
            norms.append(np.linalg.norm(phi))
        rate = (norms[-1] / norms[-101]) ** (1 / 100)
        if expect_growth:
            assert abs(rate - lam) < 1e-6
        else:
            # slowest decaying non-mean mode: |1 - 2r(1 - cos(2 pi/n))| vs pi-mode
            want = max(abs(1 - 2 * r * (1 - np.cos(2 * np.pi / n))), abs(1 - 4 * r))
            assert abs(rate - want) < 1e-6 and rate < 1


def test_three_level_growth_matches_max_root():
    """Ex.2 Case 3 scheme on D2Q9: measured asymptotic growth per step equals
    the largest root modulus of lambda^2 - p1 lambda - p0 over the grid modes."""
    case = I.random_linear_case(2, seed=9, n=(16, 16))
    a, ah = SCHEMES["ex2_case3"]
    spec = lin_spec("D2Q9", case, a, ah)
    spec["u"] = (0.9, 0.7)
    spec["K"] = [[0.02, 0.0], [0.0, 0.02]]
    E, w, pairs = O.lattice_info("D2Q9")
    _, _, tab = O.tables(spec)
    lam = S.max_amplification(E, pairs, tab["ubp"], tab["ubm"], spec["n"], a, ah)
    prev, cur = case["phim"], case["phi0"]
    logs = []
    for _ in range(1500):
        prev, cur = cur, O.mmfd_step(spec, cur, prev)
        nrm = np.linalg.norm(cur)
        logs.append(np.log(nrm))
        prev, cur = prev / nrm, cur / nrm  # linear scheme: rescaling keeps the rate
    rate = np.exp(np.mean(logs[-100:]))
    assert lam > 1.0
    assert abs(rate - lam) < 1e-4 * lam


def test_table3_stability_bracket():
    """Table 3 (Example 2, Case 1: SRT, D = 0.01, u = (1, 1), periodic [0,2)^2):
    the runs at |u|^2/c_s^2 = 50/3 and 25/6 diverge, those at 25/24 and 25/96
    stay bounded.  The exact max |lambda| over the grid's Fourier modes of the
    oracle's linear step must fall on the same sides of 1."""
    import json
    import os
    from fractions import Fraction as F
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_values.json")))
    E, w, pairs = O.lattice_info("D2Q9")
    for i, (sdx, sdt, sratio) in enumerate(gold["stability_ratio_table3"]["rows"]):
        dx, dt = F(sdx), F(sdt)
        assert 2 / ((dx / dt) ** 2 / 3) == F(sratio)  # |u|^2 / c_s^2 with u = (1, 1)
        nx = int(2 / dx)
        spec = dict(lattice="D2Q9", n=(nx, nx), dx=float(dx), dt=float(dt), u=(1.0, 1.0),
                    K=[[0.01, 0.0], [0.0, 0.01]], lambda_bar=1, a=S.preset_srt()[0])
        _, _, tab = O.tables(spec)
        lam = S.max_amplification(E, pairs, tab["ubp"], tab["ubm"], spec["n"], spec["a"], (0, 0, 0))
        if i < 2:
            assert lam > 1.5, (sratio, lam)
        else:
            assert lam < 1.0 + 1e-12, (sratio, lam)
