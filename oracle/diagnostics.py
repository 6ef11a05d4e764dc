"""Oracle global diagnostics: mass, momentum, kinetic energy, enstrophy.

Test infrastructure only (see the package docstring).

Kinetic energy and enstrophy are the quantities the paper follows in time for
its 2D benchmark (Sec. 4.1): the enstrophy is half the integral of the squared
vorticity.  Here both are reported as volume means (the paper does not
normalise by the area), vorticity by second-order central differences on the
periodic lattice, all in FP64.

Pinned by tests/test_oracle_diagnostics.py: the curl of a single Fourier mode
against its closed form Re(i (sin k) x A e^{ik.x}), the Taylor-Green
enstrophy and energy at t = 0 in closed form, totals of uniform flows and
density waves; tests/test_oracle_mutations.py plants mistakes in each
function and checks that these pins catch them.
"""
from __future__ import annotations

import numpy as np


def totals(rho, u):
    """(mass, p_x, p_y, p_z, kinetic energy) summed over the lattice, FP64."""
    mom = [float(np.sum(rho * u[d])) for d in range(u.shape[0])]
    while len(mom) < 3:
        mom.append(0.0)
    ke = float(np.sum(0.5 * rho * np.sum(u * u, axis=0)))
    return (float(np.sum(rho)), mom[0], mom[1], mom[2], ke)


def _ddx(a, axis):
    return 0.5 * (np.roll(a, -1, axis=axis) - np.roll(a, 1, axis=axis))


def vorticity(u):
    """Vorticity of u (D, nz, ny, nx): 2D returns (1,...) (w_z), 3D returns (3,...)."""
    X, Y, Z = 2, 1, 0  # array axes of x, y, z in a (nz, ny, nx) field
    if u.shape[0] == 2:
        return (_ddx(u[1], X) - _ddx(u[0], Y))[None]
    ux, uy, uz = u
    return np.stack([_ddx(uz, Y) - _ddx(uy, Z), _ddx(ux, Z) - _ddx(uz, X), _ddx(uy, X) - _ddx(ux, Y)])


def enstrophy(u):
    """Volume mean of |omega|^2 / 2."""
    w = vorticity(u)
    return float(np.mean(0.5 * np.sum(w * w, axis=0)))


def kinetic_energy_mean(rho, u):
    """Volume mean of rho |u|^2 / 2."""
    return float(np.mean(0.5 * rho * np.sum(u * u, axis=0)))
