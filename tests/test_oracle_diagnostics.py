"""Pins of the oracle's global diagnostics (CPU only): mass, momentum, kinetic
energy, vorticity and enstrophy (Sec. 4.1 follows the energy and the enstrophy,
half the integral of the squared vorticity, in time).

What fixes each function, independently of its code:
* vorticity: for one Fourier mode u = Re(A exp(i k.x)) on a periodic lattice the
  central difference along axis b multiplies the mode by i sin(k_b), so the
  discrete curl is Re(i (s x A) exp(i k.x)) with s = (sin k_x, sin k_y, sin k_z).
  Distinct wavenumbers on the three axes of a box with three different lengths,
  and a complex amplitude with every component non-zero, make every term of
  every component visible: an axis swap, a sign or a transposed term fails.
* enstrophy: the mean of |omega|^2/2 of such a mode is |s x A|^2/4; for the
  Taylor-Green fields of the workloads at t = 0 it is u0^2 sin^2(k)/2 in 2D and
  3 u0^2 sin^2(k)/8 in 3D (k = 2 pi/n), derived by hand from the same rule.
* totals and mean kinetic energy: a uniform flow gives mass rho V, momentum
  rho U V and energy rho |U|^2 V/2; a density wave cos(k x) with a uniform
  velocity sums to zero over whole periods; the Taylor-Green energy at rho = 1
  is u0^2/4 (2D) and u0^2/8 (3D) per node.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import diagnostics as OD


def fourier_mode(shape, m, amp):
    """u_a = Re(amp_a exp(i k.x)) on a (nz, ny, nx) lattice with k = 2 pi m / (nx, ny, nz); m = (mx, my, mz)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    k = 2 * np.pi * np.array(m, dtype=float) / np.array([nx, ny, nz], dtype=float)
    phase = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    u = np.stack([np.real(a * phase) for a in amp])
    return u, k, phase


AMP3 = np.array([0.3 + 0.7j, -0.5 + 0.2j, 0.4 - 0.6j])


def test_vorticity_of_a_fourier_mode_3d():
    shape = (12, 10, 8)
    u, k, phase = fourier_mode(shape, (1, 2, 3), AMP3)
    s = np.sin(k)
    w_hat = 1j * np.cross(s, AMP3)
    want = np.stack([np.real(c * phase) for c in w_hat])
    got = OD.vorticity(u)
    assert got.shape == (3,) + shape
    assert np.abs(got - want).max() <= 1e-14


def test_vorticity_of_a_fourier_mode_2d():
    shape = (1, 10, 8)
    amp = np.array([0.3 + 0.7j, -0.5 + 0.2j])
    u, k, phase = fourier_mode(shape, (1, 3, 0), amp)
    s = np.sin(k)
    want = np.real(1j * (s[0] * amp[1] - s[1] * amp[0]) * phase)
    got = OD.vorticity(u)
    assert got.shape == (1,) + shape
    assert np.abs(got[0] - want).max() <= 1e-14


def test_enstrophy_of_a_fourier_mode():
    shape = (12, 10, 8)
    u, k, _ = fourier_mode(shape, (1, 2, 3), AMP3)
    w_hat = np.cross(np.sin(k), AMP3)
    assert OD.enstrophy(u) == pytest.approx(float(np.sum(np.abs(w_hat) ** 2)) / 4, rel=1e-13)


@pytest.mark.parametrize("n", [8, 16, 64])
def test_taylor_green_enstrophy_at_t0(n):
    u0 = 0.05
    k = 2 * math.pi / n
    _, u2 = W.tgv2d(n, u0)
    assert OD.enstrophy(u2.reshape((2, 1, n, n))) == pytest.approx(u0**2 * math.sin(k) ** 2 / 2, rel=1e-12)
    _, u3 = W.tgv3d(n, u0)
    assert OD.enstrophy(u3) == pytest.approx(3 * u0**2 * math.sin(k) ** 2 / 8, rel=1e-12)


def test_totals_of_a_uniform_flow():
    shape = (4, 5, 6)
    V = 4 * 5 * 6
    rho = np.full(shape, 1.25)
    U = np.array([0.1, -0.2, 0.05])
    u = np.broadcast_to(U[:, None, None, None], (3,) + shape).copy()
    m, px, py, pz, ke = OD.totals(rho, u)
    assert m == pytest.approx(1.25 * V, rel=1e-15)
    assert (px, py, pz) == pytest.approx(tuple(1.25 * U * V), rel=1e-14)
    assert ke == pytest.approx(0.5 * 1.25 * float(U @ U) * V, rel=1e-14)
    assert OD.kinetic_energy_mean(rho, u) == pytest.approx(0.5 * 1.25 * float(U @ U), rel=1e-14)
    # 2D fields: the z momentum is reported as zero
    m2, px2, py2, pz2, ke2 = OD.totals(rho[:1], u[:2, :1])
    assert (m2, px2, py2, pz2) == pytest.approx((1.25 * 30, 1.25 * 0.1 * 30, -1.25 * 0.2 * 30, 0.0), rel=1e-14)
    assert ke2 == pytest.approx(0.5 * 1.25 * 0.05 * 30, rel=1e-14)


def test_totals_of_a_density_wave():
    """rho = 1 + a cos(2 pi x/n) with uniform u: the wave sums to zero over a period, so mass,
    momentum and energy are those of rho = 1; weighting by rho is visible on a velocity that
    varies with the same wave."""
    shape = (3, 4, 16)
    V = 3 * 4 * 16
    x = np.arange(16)
    a = 0.1
    c = np.cos(2 * np.pi * x / 16)
    rho = np.broadcast_to(1 + a * c, shape).copy()
    U = np.array([0.02, 0.03, -0.01])
    u = np.broadcast_to(U[:, None, None, None], (3,) + shape).copy()
    m, px, py, pz, ke = OD.totals(rho, u)
    assert m == pytest.approx(V, rel=1e-14)
    assert (px, py, pz) == pytest.approx(tuple(U * V), rel=1e-13)
    assert ke == pytest.approx(0.5 * float(U @ U) * V, rel=1e-13)
    # u_x = b cos(2 pi x/n): sum rho u_x = a b V/2 and sum rho u_x^2/2 = b^2 V/4 (the cos^3 term vanishes)
    b = 0.04
    u[0] = b * np.broadcast_to(c, shape)
    m, px, py, pz, ke = OD.totals(rho, u)
    assert px == pytest.approx(a * b * V / 2, rel=1e-12)
    want_ke = b**2 * V / 4 + 0.5 * float(U[1:] @ U[1:]) * V
    assert ke == pytest.approx(want_ke, rel=1e-12)


@pytest.mark.parametrize("n", [8, 32])
def test_taylor_green_energy_at_t0(n):
    u0 = 0.05
    _, u2 = W.tgv2d(n, u0)
    ones2 = np.ones((1, n, n))
    assert OD.kinetic_energy_mean(ones2, u2.reshape((2, 1, n, n))) == pytest.approx(u0**2 / 4, rel=1e-12)
    _, u3 = W.tgv3d(n, u0)
    assert OD.kinetic_energy_mean(np.ones((n, n, n)), u3) == pytest.approx(u0**2 / 8, rel=1e-12)
