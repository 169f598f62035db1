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
