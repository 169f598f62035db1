"""Pins of the oracle's theta step for Burgers' equation (Eq. (GCN)), solved
by the Picard-Jacobi iteration of oracle/implicit.py.

* theta = 1 is the explicit step of Eq. (2-2-1), bit for bit.
* The converged result satisfies Eq. (GCN) itself,
  x = A0 phi + theta L(phi) + (1 - theta) L(x), to the tolerance, with the
  increment L(y) = literal(y) - A0 y taken from the literal population sum of
  Eq. (2-2) (a form independent of the central form the iteration uses).
* The sweep count is the first chunk boundary where the stopping rule holds,
  recomputed with numpy norms from fixed-count solves.
* As theta -> 0 with a diffusive time step well beyond the explicit limit
  the solve still converges and stays bounded (the implicit part carries the
  stiffness), while the explicit step grows.
"""
import numpy as np
import pytest

from oracle import implicit as IM
from oracle import native as O


def burgers_case(lat, n, nu, dt_factor, theta):
    dx = 1.0 / n[0]
    A = 0.1
    dt = dt_factor * 0.3 * dx * dx / nu
    s = 2 * nu * dt / ((1.0 / 3.0) * dx * dx)
    a = ((s + 1) / 2, 1 - s, (s - 1) / 2)
    return dict(lattice=lat, eq="burgers", n=n, dx=dx, dt=dt, a=a, theta=theta)


def _state(spec, seed):
    rng = np.random.default_rng(seed)
    N = O.npoints(spec)
    return 0.1 * rng.uniform(-1, 1, N)


@pytest.mark.parametrize("lat,n", [("D2Q9", (17, 13)), ("D1Q3", (40,)), ("D2Q5", (12, 11))])
def test_theta_one_is_explicit(lat, n):
    spec = burgers_case(lat, n, 5e-3, 0.5, 1.0)
    phi = _state(spec, 1)
    x, k, conv = IM.theta_picard_solve(spec, phi, 1e-12, 2, 10)
    es = dict(spec)
    es.pop("theta")
    assert conv and k == 2
    assert np.array_equal(x, O.mmfd_step(es, phi))


@pytest.mark.parametrize("lat,n", [("D2Q9", (17, 13)), ("D1Q3", (40,)), ("D3Q19", (7, 6, 5))])
@pytest.mark.parametrize("theta", [0.5, 0.0])
def test_converged_step_satisfies_gcn(lat, n, theta):
    spec = burgers_case(lat, n, 5e-3, 4.0, theta)
    phi = _state(spec, 2)
    tol = 1e-10
    x, k, conv = IM.theta_picard_solve(spec, phi, tol, 3, 400)
    assert conv
    es = dict(spec)
    es.pop("theta")
    A0 = sum(spec["a"])

    def L(y):
        return O.literal_step(es, y) - A0 * y

    R = A0 * phi + theta * L(phi)
    r = x - R - (1 - theta) * L(x)
    assert np.linalg.norm(r) <= 1.01 * tol * np.linalg.norm(R) + 1e-13 * np.linalg.norm(R)
    # the stopping point
    _, dd, den = IM.picard_constants(spec)

    def ratio(kk):
        xk, _, _ = IM.theta_picard_solve(spec, phi, 1e-300, kk, kk)
        xk1, _, _ = IM.theta_picard_solve(spec, phi, 1e-300, kk - 1, kk - 1)
        return den * np.linalg.norm(xk - xk1) / np.linalg.norm(R)

    assert ratio(k) <= tol * (1 + 1e-9)
    if k > 3:
        assert ratio(k - 3) > tol * (1 - 1e-9)


def test_implicit_step_is_stable_beyond_the_explicit_limit():
    spec = burgers_case("D2Q9", (24, 24), 5e-3, 6.0, 0.0)  # dt 3x the explicit bound
    phi = _state(spec, 3)
    es = dict(spec)
    es.pop("theta")
    xi, xe = phi, phi
    for _ in range(30):
        xi, _, conv = IM.theta_picard_solve(dict(spec), xi, 1e-10, 4, 400)
        assert conv
        xe = O.mmfd_step(es, xe)
    assert np.abs(xi).max() <= np.abs(phi).max() * 1.0000001
    with np.errstate(invalid="ignore"):
        grew = not np.all(np.isfinite(xe)) or np.abs(xe).max() > 10 * np.abs(phi).max()
    assert grew


# ------------------------------------------------------------------ NSE
def nse_case(lat, n, theta, s_rho=1.6, s_j=0.9, dt=1.0):
    def fam(s):
        return ((s + 1) / 2, 1 - s, (s - 1) / 2)

    return dict(lattice=lat, eq="nse", n=n, dx=1.0, dt=dt, rho0=1.0, a=fam(s_rho), ab=fam(s_j),
                theta=theta)


def _nse_state(spec, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    return amp * rng.uniform(-1, 1, O.nfields(spec) * O.npoints(spec))


NSE_LATS = [("D2Q9", (9, 7)), ("D2Q5", (8, 6)), ("D3Q19", (5, 4, 4))]


@pytest.mark.parametrize("lat,n", NSE_LATS)
def test_nse_theta_one_is_explicit(lat, n):
    spec = nse_case(lat, n, 1.0)
    phi = _nse_state(spec, 4)
    x, k, conv = IM.theta_picard_solve(spec, phi, 1e-12, 2, 10)
    es = dict(spec)
    es.pop("theta")
    assert conv and k == 2
    assert np.array_equal(x, O.mmfd_step(es, phi))


@pytest.mark.parametrize("lat,n", NSE_LATS + [("D3Q7", (4, 4, 3)), ("D2Q5II", (6, 5))])
def test_nse_split_diagonal_is_the_step_jacobian_diagonal(lat, n):
    """dd of every field is the own-node coefficient the split moves: at rest
    (j = 0) the quadratic term has no first-order part, so the diagonal of the
    explicit step's Jacobian is A0_f - dd_f, measured here by central
    differences of the step map (exact for the linear parts up to rounding)."""
    d0 = 0.3 if lat == "D3Q7" else 1.0 / 3.0
    spec = dict(nse_case(lat, n, 0.5), d0=d0)
    es = dict(spec)
    es.pop("theta")
    consts = IM.picard_field_constants(spec)
    F = O.nfields(spec)
    N = O.npoints(spec)
    assert len(consts) == F
    base = np.zeros(F * N)
    h = 1e-4
    for f in range(F):
        for i in (0, N // 2, N - 1):
            e = np.zeros(F * N)
            e[f * N + i] = h
            jac = (O.mmfd_step(es, base + e)[f * N + i] - O.mmfd_step(es, base - e)[f * N + i]) / (2 * h)
            A0, dd, den = consts[f]
            assert dd > 0 and den == 1.0 + 0.5 * dd
            assert abs(jac - (A0 - dd)) <= 1e-9 * max(1.0, abs(A0 - dd)), (f, i, jac, A0 - dd)


@pytest.mark.parametrize("lat,n", NSE_LATS)
@pytest.mark.parametrize("theta", [0.5, 0.0])
def test_nse_converged_step_satisfies_gcn(lat, n, theta):
    """The converged NSE theta step solves Eq. (GCN) per field, with the
    increment taken from the literal population sum of Eq. (2-2) (independent
    of the central pair form the iteration runs), to the tolerance; the
    stopping point is the first chunk boundary where the rule holds."""
    spec = nse_case(lat, n, theta)
    phi = _nse_state(spec, 5)
    tol = 1e-10
    x, k, conv = IM.theta_picard_solve(spec, phi, tol, 3, 400)
    assert conv and k >= 3
    es = dict(spec)
    es.pop("theta")
    F = O.nfields(spec)
    N = O.npoints(spec)
    A0v = np.concatenate([np.full(N, c[0]) for c in IM.picard_field_constants(spec)])

    def L(y):
        return O.literal_step(es, y) - A0v * y

    R = A0v * phi + theta * L(phi)
    r = x - R - (1 - theta) * L(x)
    dens = np.concatenate([np.full(N, c[2]) for c in IM.picard_field_constants(spec)])
    # the stopping rule bounds den (x_k - x_(k-1)), the residual up to O(contraction)
    assert np.linalg.norm(r) <= 4 * tol * np.linalg.norm(R) + 1e-13 * np.linalg.norm(R)

    def ratio(kk):
        xk, _, _ = IM.theta_picard_solve(spec, phi, 1e-300, kk, kk)
        xk1, _, _ = IM.theta_picard_solve(spec, phi, 1e-300, kk - 1, kk - 1)
        return np.linalg.norm(dens * (xk - xk1)) / np.linalg.norm(R)

    assert ratio(k) <= tol * (1 + 1e-9)
    if k > 3:
        assert ratio(k - 3) > tol * (1 - 1e-9)
    assert F == 1 + O.DIMS[lat]


def test_nse_theta_conserves_mass_and_momentum():
    """On a periodic grid the explicit step keeps each field's total up to
    the factor A0 (= 1 for these coefficients); R's total is then the total
    T of phi^n, and a sweep maps an iterate of total T to
    (T + (1 - theta) dd T) / den = T, so every iterate, and the theta step,
    keeps the totals of mass and momentum (up to rounding)."""
    spec = nse_case("D2Q9", (10, 9), 0.5)
    phi = _nse_state(spec, 6)
    x, _, conv = IM.theta_picard_solve(spec, phi, 1e-12, 4, 400)
    assert conv
    N = O.npoints(spec)
    for f in range(3):
        s0, s1 = phi[f * N:(f + 1) * N].sum(), x[f * N:(f + 1) * N].sum()
        assert abs(s1 - s0) <= 1e-12 * max(1.0, np.abs(phi).sum())


# ------------------------------------------- linear CDE, exact periodic solve
def lcde_case(lat, n, theta, diff=2.0):
    dim = O.DIMS[lat]
    K = (np.eye(dim) * diff).tolist()
    u = [0.3, -0.2, 0.1][:dim]
    return dict(lattice=lat, eq="lcde", n=n, dx=1.0, dt=1.0, a=(1.0, 0.0, 0.0), u=u, K=K,
                theta=theta)


@pytest.mark.parametrize("lat,n", [("D2Q9", (16, 12)), ("D2Q5", (10, 8)), ("D1Q3", (30,)),
                                   ("D3Q19", (6, 5, 4))])
@pytest.mark.parametrize("theta", [0.5, 0.0])
def test_exact_periodic_theta_step(lat, n, theta):
    """The Fourier solve of the linear theta step satisfies
    x - (1 - theta)(S(x) - A0 x) = R with S the oracle's explicit step (so
    its symbol is the step's stencil), and equals the Jacobi solve of
    orc_theta_solve iterated to 1e-14."""
    spec = lcde_case(lat, n, theta)
    rng = np.random.default_rng(8)
    phi = rng.standard_normal(O.npoints(spec))
    x, R = IM.theta_exact_periodic(spec, phi)
    es = dict(spec)
    es.pop("theta")
    A0 = sum(spec["a"])
    r = x - (1 - theta) * (O.mmfd_step(es, x) - A0 * x) - R
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(R)
    xj, k, conv = O.theta_solve(spec, phi, 1e-14, 8, 20000)
    assert conv
    assert np.linalg.norm(xj - x) <= 1e-12 * np.linalg.norm(x)
