"""Pins of the oracle's rectangular lattices (Appendix A: a d0 per axis,
d0_a = c_s,a^2 / c_a^2, and a spacing per axis) for the linear CDE.

* The weights meet the lattice moment identities with d0 per axis:
  sum w = 1, sum w e = 0, sum w e_a e_b = d0_a delta_ab, and on the lattices
  with both axes in one velocity sum w e_a^2 e_b^2 = d0_a d0_b; equal values
  give the square tables exactly.
* The EDF of Eq. (3-3)/(3-4) with per-axis c~ and Q~ meets Eq. (3-5) in
  lattice units: sum g = A, sum e g = B, sum e e g = A diag(d0) + C.
* The linear CDE on a grid with dx != dy: one step multiplies a long
  Fourier mode along x (y) by exp(-K_xx k^2 dt - i u_x k dt) (resp. y) up to
  the scheme's O((k dx)^2) and O(dt^2) errors, so the per-axis mapping of u
  and K (u_a dt / dx_a, K_ab dt / (dx_a dx_b)) is the physical one.
"""
import numpy as np
import pytest

from oracle import native as O

RECT = [("D1Q3", (0.3,)), ("D2Q5", (0.3, 0.2)), ("D2Q9", (0.3, 0.45)),
        ("D3Q19", (0.3, 0.25, 0.2)), ("D3Q7", (0.3, 0.2, 0.25)), ("D3Q27", (0.3, 0.45, 0.6))]
BOTH_AXES = ("D2Q9", "D3Q19", "D3Q27")  # velocities with two nonzero components


@pytest.mark.parametrize("lat,d0v", RECT)
def test_rect_lattice_moments(lat, d0v):
    E, w, pairs = O.lattice_info_rect(lat, d0v)
    dim = O.DIMS[lat]
    Ed = E[:, :dim].astype(float)
    d = np.array(d0v[:dim])
    assert np.all(w > 0)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(w @ Ed, 0, atol=1e-16)
    assert np.allclose(np.einsum("j,ja,jb->ab", w, Ed, Ed), np.diag(d), atol=1e-15)
    if lat in BOTH_AXES:
        M4 = np.einsum("j,ja,jb->ab", w, Ed ** 2, Ed ** 2)
        for a in range(dim):
            for b in range(dim):
                if a != b:
                    assert abs(M4[a, b] - d[a] * d[b]) < 1e-15
    # equal d0 per axis: the square table exactly
    Es, ws, ps = O.lattice_info(lat, d0v[0])
    Er, wr, pr = O.lattice_info_rect(lat, [d0v[0]] * 3)
    assert np.array_equal(Es, Er) and np.array_equal(ws, wr) and ps == pr


def test_rect_refuses_unequal_d0_on_corner_lattices():
    for lat in ("D2Q5II", "D3Q9"):
        with pytest.raises(RuntimeError):
            O.lattice_info_rect(lat, [0.3, 0.2, 0.3])


@pytest.mark.parametrize("lat,d0v", [r for r in RECT if r[0] in BOTH_AXES] + [("D2Q5", (0.3, 0.2))])
def test_rect_edf_moment_identities(lat, d0v):
    """Eq. (3-5) in lattice units with d0 per axis (rD2Q5I: diagonal C only;
    its C_yy term leaks into the xx moment as on the square lattice, so the
    check there is C = 0 plus A and B)."""
    rng = np.random.default_rng(3)
    E, _, _ = O.lattice_info_rect(lat, d0v)
    dim = O.DIMS[lat]
    Ed = E[:, :dim].astype(float)
    d = np.array(d0v[:dim])
    for _ in range(10):
        A = rng.uniform(0.5, 1.5)
        B = rng.uniform(-0.3, 0.3, dim)
        Cm = rng.uniform(-0.2, 0.2, (dim, dim))
        Cm = 0.5 * (Cm + Cm.T)
        if lat == "D2Q5":
            Cm = np.zeros((dim, dim))
        g = O.edf_rect(lat, d0v, A, B, Cm)
        assert abs(g.sum() - A) < 1e-14
        assert np.allclose(Ed.T @ g, B, atol=1e-14)
        assert np.allclose(np.einsum("j,ja,jb->ab", g, Ed, Ed), A * np.diag(d) + Cm, atol=1e-14)


def _mode_multiplier(spec, axis, m=1):
    """One MMFD step applied to the mode exp(i k x_axis), k = 2 pi m / L:
    the complex multiplier, from the cosine and sine components."""
    n = spec["n"]
    idx = np.indices(tuple(reversed(n)))  # (..., y, x)
    coord = idx[len(n) - 1 - axis]
    th = 2 * np.pi * m * coord / n[axis]
    c, s = np.cos(th).ravel(), np.sin(th).ravel()
    oc, os_ = O.mmfd_step(spec, c), O.mmfd_step(spec, s)
    # f = Re(G e^{i th}) for input cos, Im(...) for input sin
    z = (oc + 1j * os_)
    return np.vdot(c + 1j * s, z) / np.vdot(c + 1j * s, c + 1j * s)


@pytest.mark.parametrize("axis", [0, 1])
def test_rect_lcde_mode_multiplier_is_physical(axis):
    """dx = 0.5, dy = 2 with d0 = (0.3, 0.25) and an anisotropic K: a long mode
    along either axis decays and advects at that axis' physical rate."""
    n = (512, 4) if axis == 0 else (4, 512)
    dxv = (0.5, 2.0)
    K = [[0.7, 0.0], [0.0, 0.2]]
    u = (0.3, -0.4)
    L = n[axis] * dxv[axis]
    k = 2 * np.pi / L
    dt = 0.05 * dxv[axis] ** 2 / max(K[0][0], K[1][1])
    # lambda_bar = 1: the u u term of C cancels the dt u u / 2 numerical
    # diffusion of the first-order time level (Eq. (TforMMFD-0))
    spec = dict(lattice="D2Q9", eq="lcde", n=n, dt=dt, dxv=dxv, d0v=(0.3, 0.25), u=u, K=K,
                a=(1.0, 0.0, 0.0), lambda_bar=1)
    G = _mode_multiplier(spec, axis)
    want = np.exp(-K[axis][axis] * k * k * dt - 1j * u[axis] * k * dt)
    rate, rate_want = -np.log(abs(G)) / dt, K[axis][axis] * k * k
    phase, phase_want = -np.angle(G) / dt, u[axis] * k
    assert abs(rate / rate_want - 1) < 3e-3, (rate, rate_want)
    assert abs(phase / phase_want - 1) < 3e-3, (phase, phase_want)
    assert abs(G - want) < 1e-6


def test_rect_equal_axes_is_the_square_step():
    """dx and d0 equal on every axis: the rectangular step equals the square
    one to rounding (the linear term is formed per axis instead of once)."""
    rng = np.random.default_rng(4)
    base = dict(lattice="D2Q9", eq="lcde", n=(12, 9), dx=0.5, dt=0.01, u=(0.3, -0.2),
                K=[[0.5, 0.1], [0.1, 0.4]], a=(1.0, 0.0, 0.0), lambda_bar=1)
    phi = rng.standard_normal(108)
    sq = O.mmfd_step(base, phi)
    rc = O.mmfd_step(dict(base, dxv=(0.5, 0.5), d0v=(1 / 3, 1 / 3)), phi)
    assert np.allclose(rc, sq, rtol=0, atol=1e-14 * np.abs(phi).max())
