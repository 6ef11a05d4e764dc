"""Von Neumann linear stability analysis of the regularised scheme (Sec. 3.6).

Test infrastructure only (see the package docstring).

The collision Omega_i(f) = f0_i + (1 - 1/tau) f1_i is linearised about a
uniform state: Lambda_ij = d Omega_i / d f_j at f = f0(rho, u) (Eq. lin1).
Plane waves exp(i k.x) turn the linear update into the q x q amplification
matrix A^-1 Lambda with A^-1 = diag(exp(-i k.xi_j)) (Eq. lin2); its
eigenvalues lambda give omega = i log lambda, so Im(omega) = ln|lambda| and a
mode grows when |lambda| > 1.

Lambda is computed by complex-step differentiation of the oracle collision
(the collision is a rational function of f, so the complex step is exact to
rounding); the eigenvalues come from numpy's LAPACK binding (Sec. 3.6
computes them numerically with a linear-algebra library too).
"""
from __future__ import annotations

import numpy as np

from . import rr
from .lattice import lattice


def jacobian(lat, N, tau, rho, u, h=1e-30, n1=None):
    """Lambda = dOmega/df at the equilibrium with density rho and velocity u (f1 at order n1,
    default ``rr.f1_order``)."""
    L = lattice(lat) if isinstance(lat, str) else lat
    u = np.asarray(u, dtype=float).reshape(L.D)
    fbar = rr.init_populations(L, N, np.array(rho, dtype=float), u)
    q = L.q
    J = np.zeros((q, q))
    for j in range(q):
        fc = fbar.astype(complex)
        fc[j] += 1j * h
        J[:, j] = np.imag(rr.collide(L, N, tau, fc, n1)) / h
    return J


def amplification_eigs(lat, N, tau, rho, u, kx, ky, kz=None, n1=None):
    """Eigenvalues of A^-1 Lambda for every wavevector of the given grids.

    kx, ky (and kz for 3D) are broadcastable arrays; returns (..., q) complex.
    """
    L = lattice(lat) if isinstance(lat, str) else lat
    J = jacobian(L, N, tau, rho, u, n1=n1)
    kx, ky = np.broadcast_arrays(np.asarray(kx, float), np.asarray(ky, float))
    kz = np.zeros_like(kx) if kz is None else np.broadcast_to(np.asarray(kz, float), kx.shape)
    c = L.c.astype(float)
    phase = np.exp(-1j * (kx[..., None] * c[:, 0] + ky[..., None] * c[:, 1] + kz[..., None] * c[:, 2]))
    M = phase[..., :, None] * J[None, :, :] if kx.ndim == 0 else phase[..., :, None] * J
    return np.linalg.eigvals(M)


def max_growth(lat, N, tau, rho, u, nk=64):
    """max over the k-grid [-pi, pi)^2 (k_z = 0) and modes of ln|lambda| = Im(omega)."""
    k = -np.pi + 2 * np.pi * np.arange(nk) / nk
    KX, KY = np.meshgrid(k, k, indexing="ij")
    lam = amplification_eigs(lat, N, tau, rho, u, KX, KY)
    return float(np.log(np.abs(lam)).max())


def dissipation_kx(lat, N, tau, rho, u, kx):
    """Im(omega_j) for k = (kx, 0): array (len(kx), q), sorted per kx."""
    lam = amplification_eigs(lat, N, tau, rho, u, np.asarray(kx), np.zeros_like(kx))
    return np.sort(np.log(np.abs(lam)), axis=-1)
