"""Seeded synthetic workloads for the MesoFD / MMFD time step.

This module holds only input recipes: grid sizes, physical parameters and
seeded initial fields.  It contains none of the method's arithmetic (no EDF,
no coefficient mapping, no update rule), so both the GPU library's callers and
the FP64 oracle's tests may draw from it.

State conventions (lattice units, c = dx/dt):
* scalar NCDE (linear CDE, Burgers): one field phi;
* NSE: fields (rho - rho0, j_x, j_y[, j_z]) with j = rho u dt/dx.
Arrays are float64, field-major ``[field][z][y][x]``, flattened.
"""
from __future__ import annotations

import math

import numpy as np


def _grid(n, length=1.0):
    """Node coordinates x_i = i * dx (vertex-centred, periodic)."""
    dx = length / n
    return np.arange(n, dtype=np.float64) * dx, dx


# ----------------------------------------------------------------- linear CDE

def c1_linear_1d(n=1024, seed=1):
    """1D linear CDE, D1Q3, periodic, N nodes on [0,1): u=0.1, D=0.01,
    dt = 0.5 * min(dx^2/(2D), 2D/u^2) = 25 * 2^-20 at N = 1024,
    phi0 = sin(2 pi x) + U(-1e-3, 1e-3)."""
    x, dx = _grid(n)
    D, u = 0.01, 0.1
    dt = 0.5 * min(dx * dx / (2 * D), 2 * D / (u * u))
    if n == 1024:
        dt = 25.0 * 2.0 ** -20
    rng = np.random.default_rng(seed)
    phi0 = np.sin(2 * np.pi * x) + rng.uniform(-1e-3, 1e-3, n)
    return dict(lattice="D1Q3", n=(n,), dx=dx, dt=dt, u=(u,), K=[[D]], D=D,
                lambda_bar=0, steps=1000, phi0=phi0)


C2_K = [[0.02, 0.005], [0.005, 0.01]]
C2_U = (0.05, 0.03)


def c2_hill_2d(n=2048, seed=2, sigma=0.05, noise=1e-4):
    """2D anisotropic linear CDE on [0,1)^2, D2Q9, periodic n x n.
    dt = 16 dx^2 (= 2^-18 at n = 2048), lambda_bar = 1,
    phi0 = Gaussian hill at (1/2, 1/2) (torus distance) + U(-noise, noise)."""
    x, dx = _grid(n)
    dt = 16.0 * dx * dx
    rng = np.random.default_rng(seed)
    dxs = np.minimum(np.abs(x - 0.5), 1.0 - np.abs(x - 0.5))
    r2 = dxs[None, :] ** 2 + dxs[:, None] ** 2
    phi0 = np.exp(-r2 / (2 * sigma * sigma)) + rng.uniform(-noise, noise, (n, n))
    return dict(lattice="D2Q9", n=(n, n), dx=dx, dt=dt, u=C2_U, K=C2_K, lambda_bar=1,
                steps=10000, phi0=phi0.ravel())


def gaussian_hill_exact(n, t, sigma=0.05, K=C2_K, u=C2_U, images=1):
    """Exact solution of the linear CDE for the Gaussian hill (periodic
    images summed): sigma^2/sqrt(det S_t) exp(-r^T S_t^-1 r / 2),
    S_t = sigma^2 I + 2 K t, r = x - x0 - u t."""
    x, _ = _grid(n)
    S = sigma * sigma * np.eye(2) + 2.0 * np.asarray(K) * t
    Si = np.linalg.inv(S)
    X, Y = np.meshgrid(x, x, indexing="xy")
    out = np.zeros((n, n))
    for ix in range(-images, images + 1):
        for iy in range(-images, images + 1):
            rx = X - 0.5 - u[0] * t + ix
            ry = Y - 0.5 - u[1] * t + iy
            q = Si[0, 0] * rx * rx + 2 * Si[0, 1] * rx * ry + Si[1, 1] * ry * ry
            out += np.exp(-0.5 * q)
    return out * sigma * sigma / math.sqrt(np.linalg.det(S))


def example1_source_2d(n=2048, kappa=0.01, u=(0.1, 0.1)):
    """Example 1 of the paper (isotropic CDE with a source), D2Q9, periodic
    [0,2)^2 with n nodes a side: dx = 2/n, the example's diffusive scaling
    N_t = 0.06 N_x^2 (N_x = 1/dx) read as dt = dx^2 / 0.06, u = (0.1, 0.1),
    kappa = 0.01.  The source is R = exp(lam t) G(x, y) with
    lam = 1 - 2 pi^2 kappa, G = sin(pi (x + y)) + pi (u_x + u_y) cos(pi (x + y));
    the exact solution is exp(lam t) sin(pi (x + y)).  Returns the grid, the
    physical parameters, G and the exact fields at t = 0 and t = -dt."""
    x, dx = _grid(n, 2.0)
    dt = dx * dx / 0.06
    X, Y = np.meshgrid(x, x)
    lam = 1.0 - 2.0 * math.pi ** 2 * kappa
    G = (np.sin(math.pi * (X + Y)) + math.pi * (u[0] + u[1]) * np.cos(math.pi * (X + Y))).ravel()
    exact = lambda t: math.exp(lam * t) * np.sin(math.pi * (X + Y)).ravel()
    return dict(n=(n, n), dx=dx, dt=dt, u=tuple(u), K=[[kappa, 0.0], [0.0, kappa]], lam=lam,
                G=G, phi0=exact(0.0), phim=exact(-dt), exact=exact)


def random_linear_case(dim, seed, n=None):
    """Random anisotropic linear CDE on a small periodic grid (for pins)."""
    rng = np.random.default_rng(seed)
    n = n or {1: (23,), 2: (13, 11), 3: (7, 6, 5)}[dim]
    u = rng.uniform(-0.4, 0.4, dim)
    A = rng.uniform(-0.3, 0.3, (dim, dim))
    K = 0.5 * np.eye(dim) + 0.1 * (A @ A.T)
    return dict(n=n, dx=1.0, dt=1.0, u=tuple(u), K=K.tolist(),
                phi0=rng.standard_normal(int(np.prod(n))),
                phim=rng.standard_normal(int(np.prod(n))))


# ------------------------------------------------------------------- Burgers

def burgers_instance(rng, side_lo=64, side_hi=1024, steps_lo=500, steps_hi=5000, A=0.1):
    """One 2D Burgers NCDE instance (flux phi^2/2 per axis) on [0,1)^2:
    side log-uniform, nu ~ U[1e-3, 1e-2], steps ~ U{lo..hi},
    dt = 0.5 * min(0.3 dx^2 / nu, nu / A^2),
    phi0 = A sin(2 pi k1 x + t1) sin(2 pi k2 y + t2) + A 1e-3 U(-1,1)."""
    side = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
    nu = float(rng.uniform(1e-3, 1e-2))
    steps = int(rng.integers(steps_lo, steps_hi + 1))
    k1, k2 = (int(v) for v in rng.integers(1, 5, 2))
    t1, t2 = (float(v) for v in rng.uniform(0, 2 * np.pi, 2))
    x, dx = _grid(side)
    dt = 0.5 * min(0.3 * dx * dx / nu, nu / (A * A))
    phi0 = (A * np.sin(2 * np.pi * k1 * x[None, :] + t1) * np.sin(2 * np.pi * k2 * x[:, None] + t2)
            + A * 1e-3 * rng.uniform(-1, 1, (side, side)))
    return dict(lattice="D2Q9", eq="burgers", n=(side, side), dx=dx, dt=dt, nu=nu,
                steps=steps, phi0=phi0.ravel())


def c4_batch(count=256, seed=4, **kw):
    rng = np.random.default_rng(seed)
    return [burgers_instance(rng, **kw) for _ in range(count)]


# ----------------------------------------------------------------------- NSE

def tgv_2d(n=4096, seed=3, U0=1.0, rho0=1.0, nu=0.01, courant=0.05, noise=1e-4):
    """2D Taylor-Green vortex on [0, 2 pi)^2, Re = U0/(k nu) with k = 1:
    u = -U0 cos x sin y, v = U0 sin x cos y,
    rho = rho0 - rho0 U0^2 (cos 2x + cos 2y) / (4 c_s^2), c_s^2 = (dx/dt)^2/3,
    dt = courant dx / U0, velocity noise U(-noise, noise) U0 per component.
    State: (rho - rho0, j_x, j_y), j = rho u dt/dx."""
    x, dx = _grid(n, 2 * np.pi)
    dt = courant * dx / U0
    cs2 = (dx / dt) ** 2 / 3.0
    X, Y = np.meshgrid(x, x, indexing="xy")
    rng = np.random.default_rng(seed)
    u = -U0 * np.cos(X) * np.sin(Y) + noise * U0 * rng.uniform(-1, 1, (n, n))
    v = U0 * np.sin(X) * np.cos(Y) + noise * U0 * rng.uniform(-1, 1, (n, n))
    drho = -rho0 * U0 * U0 * (np.cos(2 * X) + np.cos(2 * Y)) / (4 * cs2)
    rho = rho0 + drho
    s = dt / dx
    state = np.concatenate([drho.ravel(), (rho * u * s).ravel(), (rho * v * s).ravel()])
    return dict(lattice="D2Q9", eq="nse", n=(n, n), dx=dx, dt=dt, nu=nu, rho0=rho0,
                U0=U0, steps=20000, state0=state)


def tgv_2d_exact_velocity(n, t, U0=1.0, nu=0.01):
    """Incompressible TGV velocity at time t: amplitude decays as exp(-2 nu t)."""
    x, _ = _grid(n, 2 * np.pi)
    X, Y = np.meshgrid(x, x, indexing="xy")
    f = math.exp(-2 * nu * t)
    return -U0 * np.cos(X) * np.sin(Y) * f, U0 * np.sin(X) * np.cos(Y) * f


def tgv_3d(n=512, seed=3, U0=1.0, rho0=1.0, nu=None, courant=0.05, noise=1e-4, dtype=np.float64):
    """3D Taylor-Green vortex on [0, 2 pi)^3:
    u = U0 (sin x cos y cos z, -cos x sin y cos z, 0),
    p = rho0 U0^2/16 (cos 2x + cos 2y)(cos 2z + 2), rho = rho0 + p / c_s^2.
    Default nu from lattice viscosity 0.04074 at courant 0.05 (nu = 0.04074 dx^2/dt).
    Built by broadcasting 1D factors (no full coordinate grids)."""
    x, dx = _grid(n, 2 * np.pi)
    dt = courant * dx / U0
    cs2 = (dx / dt) ** 2 / 3.0
    if nu is None:
        nu = 0.04074 * dx * dx / dt
    sx, cx = np.sin(x).astype(dtype), np.cos(x).astype(dtype)
    c2 = np.cos(2 * x).astype(dtype)
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    s = dt / dx
    p = (rho0 * U0 * U0 / 16.0) * (c2[None, None, :] + c2[None, :, None]) * (c2[:, None, None] + 2.0)
    drho = (p / cs2).astype(dtype)
    del p
    rho = rho0 + drho
    u = (U0 * sx[None, None, :] * cx[None, :, None] * cx[:, None, None]
         + (noise * U0) * rng.uniform(-1, 1, shape).astype(dtype))
    ju = (rho * u * s).astype(dtype)
    del u
    v = (-U0 * cx[None, None, :] * sx[None, :, None] * cx[:, None, None]
         + (noise * U0) * rng.uniform(-1, 1, shape).astype(dtype))
    jv = (rho * v * s).astype(dtype)
    del v
    jw = (rho * ((noise * U0) * rng.uniform(-1, 1, shape).astype(dtype)) * s).astype(dtype)
    state = np.concatenate([drho.ravel(), ju.ravel(), jv.ravel(), jw.ravel()])
    return dict(lattice="D3Q19", eq="nse", n=(n, n, n), dx=dx, dt=dt, nu=nu, rho0=rho0,
                U0=U0, steps=1000, state0=state)


# ------------------------------------------------------------------- serving

def serving_trace(count=2000, warmup=200, rate=200.0, seed=5, side_lo=128, side_hi=2048,
                  steps_lo=100, steps_hi=5000, nse_fraction=0.5):
    """Poisson arrivals of mixed 2D Burgers / 2D NSE (TGV) MMFD solves:
    side and steps log-uniform, type Bernoulli(nse_fraction).  Returns a list of
    request descriptors (the initial fields are generated per request from
    `seed` so that a request can be rebuilt identically)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count + warmup):
        t += rng.exponential(1.0 / rate)
        side = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
        steps = int(round(math.exp(rng.uniform(math.log(steps_lo), math.log(steps_hi)))))
        kind = "nse" if rng.uniform() < nse_fraction else "burgers"
        out.append(dict(id=i, arrival=t, side=side, steps=steps, kind=kind,
                        seed=int(rng.integers(0, 2 ** 31 - 1)), warmup=i < warmup))
    return out


def serving_request_state(req, A=0.1):
    """Initial state and parameters of one serving request."""
    rng = np.random.default_rng(req["seed"])
    if req["kind"] == "burgers":
        inst = burgers_instance(rng, side_lo=req["side"], side_hi=req["side"],
                                steps_lo=req["steps"], steps_hi=req["steps"], A=A)
        return inst
    inst = tgv_2d(n=req["side"], seed=req["seed"])
    inst["steps"] = req["steps"]
    return inst
