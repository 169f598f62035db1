"""Convergence of the oracle to analytic solutions (second order in the
diffusive scaling dt ~ dx^2), which pins the PDE-coefficient mapping:
alpha = -(A22/A10) dt beta c_s^2 for the CDE, the Burgers flux scaling, and
nu = -(A22/A10) dt c_s^2 for the NSE.

* 1D linear CDE, decaying sinusoid (the C1 workload's equation);
* 2D anisotropic linear CDE, Gaussian hill (the C2 workload's equation);
* 2D Burgers NCDE on the diagonal, exact by the Cole-Hopf transform;
* 2D NSE, Taylor-Green vortex, three-level TRT scheme.
"""
import math

import numpy as np
import pytest
from scipy.special import ive

import mfd_inputs as I
from oracle import native as O
from oracle import scheme as S

THIRD = 1.0 / 3.0


def order(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_c1_sinusoid_second_order():
    D, u, T = 0.01, 0.1, 0.25
    errs = []
    for n in (32, 64, 128):
        dx = 1.0 / n
        r = 0.25
        dt = r * dx * dx / D
        steps = int(round(T / dt))
        dt = T / steps
        s = S.two_level_s_for(D, dx, dt, THIRD)
        spec = dict(lattice="D1Q3", n=(n,), dx=dx, dt=dt, u=(u,), K=[[D]], a=S.preset_two_level(s)[0])
        x = np.arange(n) * dx
        phi = np.sin(2 * np.pi * x)
        for _ in range(steps):
            phi = O.mmfd_step(spec, phi)
        ex = math.exp(-4 * math.pi ** 2 * D * T) * np.sin(2 * np.pi * (x - u * T))
        errs.append(np.abs(phi - ex).max())
    for p in order(errs):
        assert 1.8 < p < 2.2, errs


def test_c2_gaussian_hill_second_order():
    T = 0.0625  # dt = 16 dx^2 divides T on every grid
    errs = []
    for n in (32, 64, 128):
        cfg = I.c2_hill_2d(n=n, noise=0.0, sigma=0.1)
        steps = int(round(T / cfg["dt"]))
        assert steps * cfg["dt"] == T
        spec = dict(lattice="D2Q9", n=cfg["n"], dx=cfg["dx"], dt=cfg["dt"], u=cfg["u"], K=cfg["K"],
                    lambda_bar=1, a=S.preset_srt()[0])
        phi = cfg["phi0"]
        for _ in range(steps):
            phi = O.mmfd_step(spec, phi)
        ex = I.gaussian_hill_exact(n, T, sigma=0.1)
        errs.append(np.abs(phi - ex.ravel()).max())
    for p in order(errs):
        assert 1.8 < p < 2.3, errs


def burgers_cole_hopf(s, t, W, mu, mmax=60):
    """w_t + w w_s = mu w_ss, w(s,0) = W sin(2 pi s), 1-periodic:
    w = -2 mu theta_s / theta with theta = I0(z) + 2 sum I_m(z) e^{-4 pi^2 m^2 mu t} cos(2 pi m s),
    z = W / (4 pi mu)."""
    z = W / (4 * math.pi * mu)
    th = np.full_like(s, ive(0, z))
    ths = np.zeros_like(s)
    for m in range(1, mmax):
        c = 2 * ive(m, z) * math.exp(-4 * math.pi ** 2 * m * m * mu * t)
        th += c * np.cos(2 * math.pi * m * s)
        ths += -c * 2 * math.pi * m * np.sin(2 * math.pi * m * s)
    return -2 * mu * ths / th


def test_burgers_diagonal_cole_hopf():
    """phi(x,y,t) = g(x+y,t) with g_t + 2 g g_s = 2 nu g_ss: w = 2g solves
    viscous Burgers with mu = 2 nu."""
    nu, A, s_par = 0.02, 0.5, 0.6
    T = 5.0 / 64.0
    errs = []
    for n in (32, 64, 128):
        dx = 1.0 / n
        dt = s_par * THIRD * dx * dx / (2 * nu)
        steps = int(round(T / dt))
        assert abs(steps * dt - T) < 1e-12
        s = S.two_level_s_for(nu, dx, dt, THIRD)
        spec = dict(lattice="D2Q9", eq="burgers", n=(n, n), dx=dx, dt=dt, a=S.preset_two_level(s)[0])
        x = np.arange(n) * dx
        sxy = x[None, :] + x[:, None]
        phi = (A * np.sin(2 * np.pi * sxy)).ravel()
        for _ in range(steps):
            phi = O.mmfd_step(spec, phi)
        ex = 0.5 * burgers_cole_hopf(sxy, T, 2 * A, 2 * nu)
        errs.append(np.abs(phi - ex.ravel()).max())
    for p in order(errs):
        assert 1.8 < p < 2.3, errs


@pytest.mark.parametrize("form", ["mmfd", "mesofd"])
def test_tgv_three_level_trt(form):
    """TRT three-level MMFD for the NSE converges to the incompressible
    Taylor-Green vortex in the diffusive scaling (Mach ~ dx)."""
    nu, U0, nuh = 0.05, 0.1, 0.1
    errs = []
    for n in (16, 32, 64):
        dx = 2 * math.pi / n
        dt = nuh * dx * dx / nu
        steps = (n // 16) ** 2 * 8
        T = steps * dt
        cfg = I.tgv_2d(n=n, U0=U0, nu=nu, courant=U0 * dt / dx, noise=0.0)
        assert abs(cfg["dt"] - dt) < 1e-14 * dt
        s = S.trt_s_for(nu, dx, dt, THIRD)
        a, ah = S.preset_trt(s)
        spec = dict(lattice="D2Q9", eq="nse", n=(n, n), dx=dx, dt=dt, rho0=1.0, a=a, ah=ah, levels=3)
        cur = cfg["state0"]
        prev = cur.copy()
        N = n * n
        if form == "mmfd":
            for _ in range(steps):
                prev, cur = cur, O.mmfd_step(spec, cur, prev)
        else:
            pop = O.init_populations(spec, cur)
            for _ in range(steps):
                pop, prev = O.mesofd_step(spec, pop, prev)
            cur = O.moments(spec, pop)
        rho = 1.0 + cur[:N]
        ux = cur[N:2 * N] / rho * dx / dt
        uy = cur[2 * N:] / rho * dx / dt
        exu, exv = I.tgv_2d_exact_velocity(n, T, U0=U0, nu=nu)
        errs.append(max(np.abs(ux - exu.ravel()).max(), np.abs(uy - exv.ravel()).max()) / U0)
    # pre-asymptotic acoustic transients of the weakly compressible start give
    # observed orders 3.1 then 1.5 (1.7 at 128^2); a wrong viscosity mapping
    # would stall the error at O(1e-2) instead
    for p in order(errs):
        assert p > 1.3, errs
    assert errs[-1] < 1e-3
