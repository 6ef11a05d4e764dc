"""Seeded synthetic inputs shared by the tests, the oracle runs and bench.py.

This module holds no lattice Boltzmann arithmetic: it only produces initial
density / velocity / stress fields (float64 numpy arrays, layout [d][z][y][x],
x fastest) and raw random numbers.  Both sides (the FP64 oracle and the HIP
library) build their own populations from these fields.

Flow recipes: the dipole of the paper's dipole-wall benchmark (Sec. 4.1, a
closed box), and periodic stand-ins for its other flows: Taylor--Green
vortices, a double shear layer, random divergence-free fields and decaying 2D
turbulence, at the Reynolds / Mach numbers of the workload table below.
"""
from __future__ import annotations

import math

import numpy as np

CS = 1.0 / math.sqrt(3.0)  # lattice sound speed used to convert Mach numbers to velocities


def tgv2d(n, u0):
    """2D Taylor--Green vortex, wavelength = box: rho (1,n,n), u (2,1,n,n)."""
    k = 2.0 * math.pi / n
    x = np.arange(n, dtype=float)
    X, Y = np.meshgrid(x, x, indexing="xy")  # X varies along the last axis
    ux = -u0 * np.cos(k * X) * np.sin(k * Y)
    uy = u0 * np.sin(k * X) * np.cos(k * Y)
    rho = 1.0 - 0.75 * u0 * u0 * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    return rho[None], np.stack([ux, uy])[:, None]


def tgv3d(n, u0):
    """3D Taylor--Green vortex: rho (n,n,n), u (3,n,n,n)."""
    k = 2.0 * math.pi / n
    x = np.arange(n, dtype=float)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    ux = u0 * np.sin(k * X) * np.cos(k * Y) * np.cos(k * Z)
    uy = -u0 * np.cos(k * X) * np.sin(k * Y) * np.cos(k * Z)
    uz = np.zeros_like(ux)
    rho = 1.0 + (3.0 * u0 * u0 / 16.0) * (np.cos(2 * k * X) + np.cos(2 * k * Y)) * (np.cos(2 * k * Z) + 2.0)
    return rho, np.stack([ux, uy, uz])


def shear_layer(n, u0, seed, width_frac=1.0 / 80.0, pert=0.05):
    """Doubly periodic double shear layer on an n x n box: rho (1,n,n), u (2,1,n,n)."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    delta = n * width_frac
    x = np.arange(n, dtype=float)
    X, Y = np.meshgrid(x, x, indexing="xy")
    ux = np.where(Y <= n / 2, u0 * np.tanh((Y - n / 4) / delta), u0 * np.tanh((3 * n / 4 - Y) / delta))
    uy = pert * u0 * np.sin(2 * math.pi * X / n + phi)
    return np.ones((1, n, n)), np.stack([ux, uy])[:, None]


def random_solenoidal3d(n, kmax, urms, seed, kmin=1.0, shape=None):
    """Random divergence-free velocity with a flat spectrum for kmin <= |k| <= kmax.

    shape = (nz, ny, nx) overrides the cubic box.  Returns rho (ones), u (3,nz,ny,nx),
    scaled so that the rms of |u| equals ``urms``.
    """
    nz, ny, nx = shape if shape is not None else (n, n, n)
    rng = np.random.default_rng(seed)
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.rfftfreq(nx) * nx
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    k2 = KX**2 + KY**2 + KZ**2
    band = (k2 >= kmin**2) & (k2 <= kmax**2)
    g = rng.standard_normal((3,) + k2.shape) + 1j * rng.standard_normal((3,) + k2.shape)
    g *= band
    kvec = np.stack([KX, KY, KZ])
    safe = np.where(k2 > 0, k2, 1.0)
    g = g - kvec * (np.sum(kvec * g, axis=0) / safe)  # project out the longitudinal part
    u = np.stack([np.fft.irfftn(g[d], s=(nz, ny, nx), axes=(0, 1, 2)) for d in range(3)])
    u *= urms / math.sqrt(np.mean(np.sum(u**2, axis=0)))
    return np.ones((nz, ny, nx)), u


def random_vorticity2d(n, kmin, kmax, urms, seed):
    """Decaying-turbulence start: random-phase vorticity with flat amplitude on kmin <= |k| <= kmax.

    Returns rho (1,n,n) ones and u (2,1,n,n) from the streamfunction, rms|u| = urms.
    """
    rng = np.random.default_rng(seed)
    k = np.fft.fftfreq(n) * n
    KY, KX = np.meshgrid(k, k, indexing="ij")
    k2 = KX**2 + KY**2
    band = (k2 >= kmin**2) & (k2 <= kmax**2)
    w_hat = np.exp(2j * math.pi * rng.uniform(size=(n, n))) * band
    w = np.real(np.fft.ifft2(w_hat))
    w_hat = np.fft.fft2(w)  # Hermitian-symmetric after taking the real part
    psi_hat = np.where(k2 > 0, w_hat / np.where(k2 > 0, k2, 1.0), 0.0)
    scale = 2 * math.pi / n
    ux = np.real(np.fft.ifft2(1j * KY * scale * psi_hat))
    uy = np.real(np.fft.ifft2(-1j * KX * scale * psi_hat))
    u = np.stack([ux, uy])
    u *= urms / math.sqrt(np.mean(np.sum(u**2, axis=0)))
    return np.ones((1, n, n)), u[:, None]


def dipole(n_unit, omega_e=299.5286, r0=0.1, centres=((0.0, 0.1), (0.0, -0.1))):
    """Dipole of the dipole-wall benchmark (Sec. 4.1, Eqs. dipole1 / dipole2) in the box [-1, 1]^2.

    Nodes at x = -1 + i / n_unit, i = 0 .. 2 n_unit (the walls lie on the first and last node).
    Returns the velocity in the paper's dimensionless units, u (2, 1, m, m), m = 2 n_unit + 1,
    exactly 0 on the wall nodes, and the node coordinate x (m,)."""
    m = 2 * n_unit + 1
    x = -1.0 + np.arange(m, dtype=float) / n_unit
    X, Y = np.meshgrid(x, x, indexing="xy")
    (x1, y1), (x2, y2) = centres
    e1 = np.exp(-((X - x1) ** 2 + (Y - y1) ** 2) / r0**2)
    e2 = np.exp(-((X - x2) ** 2 + (Y - y2) ** 2) / r0**2)
    ux = -0.5 * abs(omega_e) * (Y - y1) * e1 + 0.5 * abs(omega_e) * (Y - y2) * e2
    uy = 0.5 * abs(omega_e) * (X - x1) * e1 - 0.5 * abs(omega_e) * (X - x2) * e2
    u = np.stack([ux, uy])[:, None]
    u[:, :, [0, -1], :] = 0.0
    u[:, :, :, [0, -1]] = 0.0
    return u, x


def smooth_random(ncomp, shape, amp, seed, kmax=2):
    """Smooth random periodic fields: a few low Fourier modes, max |value| about ``amp``."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((ncomp,) + tuple(shape))
    for c in range(ncomp):
        for _ in range(4):
            kx, ky = rng.integers(-kmax, kmax + 1, size=2)
            kz = rng.integers(-kmax, kmax + 1) if nz > 1 else 0
            ph = rng.uniform(0, 2 * math.pi)
            out[c] += rng.uniform(-1, 1) * np.cos(2 * math.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
    return amp * out / 4.0


def noise(shape, amp, seed):
    """Independent normal deviates of standard deviation ``amp``."""
    return amp * np.random.default_rng(seed).standard_normal(shape)


# Workload table.  Relaxation times were computed once from the stated Reynolds
# number with the lattice viscosity nu = (tau - 1/2)/3 and are written out as
# numbers here.
WORKLOADS = {
    # 64^2 TGV, u0 = 0.05, Re = u0*64/nu = 100 -> nu = 0.032, tau = 0.596
    "tgv2d_64": dict(lattice="D2Q9", order=4, n=64, u0=0.05, tau=0.596, steps=1000),
    # 2048^2 double shear layer, Re = u0*L/nu = 1e4
    "shear_2048_ma02": dict(lattice="D2Q9", order=4, n=2048, u0=0.2 * CS, tau=0.570945, steps=20000),
    "shear_2048_ma05": dict(lattice="D2Q9", order=4, n=2048, u0=0.5 * CS, tau=0.677362, steps=20000),
    # 256^3 TGV, Re = u0*(N/2pi)/nu = 1600
    "tgv3d_256_ma01": dict(lattice="D3Q27", order=4, n=256, u0=0.1 * CS, tau=0.504411, steps=10000),
    "tgv3d_256_ma05": dict(lattice="D3Q27", order=4, n=256, u0=0.5 * CS, tau=0.522053, steps=10000),
    # same flows at 64^3 for the oracle-side curves (same convective time in 2500 steps)
    "tgv3d_64_ma01": dict(lattice="D3Q27", order=4, n=64, u0=0.1 * CS, tau=0.501103, steps=2500),
    "tgv3d_64_ma05": dict(lattice="D3Q27", order=4, n=64, u0=0.5 * CS, tau=0.505513, steps=2500),
    # 512^3 random solenoidal field, |k| <= 8, rms Ma 0.1, tau = 0.51
    # D3Q19 at order 4 with f1 stopping at order 3, the reading that is stable at rest at this tau
    # (with f1 at order 4 the model grew high-wavenumber modes at rest, 0.0285 per step)
    "solenoidal_512_d3q19": dict(lattice="D3Q19", order=4, n=512, kmax=8, urms=0.1 * CS, tau=0.51, steps=1000),
    "solenoidal_512_d3q27": dict(lattice="D3Q27", order=4, n=512, kmax=8, urms=0.1 * CS, tau=0.51, steps=1000),
    # decaying 2D turbulence for the learned closure: fine 1024^2, coarse 256^2 (dx_c = 4 dx_f)
    "turb2d_fine_1024": dict(lattice="D2Q9", order=4, n=1024, kmin=4, kmax=12, urms=0.1 * CS, tau=0.535472),
    "turb2d_coarse_256": dict(lattice="D2Q9", order=4, n=256, tau=0.508868),
}


def initial_fields(name, seed=0):
    """rho (nz,ny,nx) and u (d,nz,ny,nx) at t = 0 of the workload ``name`` of WORKLOADS, with the
    box shape (nz, ny, nx); the same recipes the full-size tests use."""
    cfg = WORKLOADS[name]
    n = cfg["n"]
    if name.startswith("tgv2d"):
        rho, u = tgv2d(n, cfg["u0"])
    elif name.startswith("shear"):
        rho, u = shear_layer(n, cfg["u0"], seed)
    elif name.startswith("tgv3d"):
        rho, u = tgv3d(n, cfg["u0"])
    elif name.startswith("solenoidal"):
        rho, u = random_solenoidal3d(n, cfg["kmax"], cfg["urms"], seed)
    elif name.startswith("turb2d_fine"):
        rho, u = random_vorticity2d(n, cfg["kmin"], cfg["kmax"], cfg["urms"], seed)
    else:
        raise KeyError(f"{name} has no initial-field recipe of its own")
    shape = (1, n, n) if cfg["lattice"] == "D2Q9" else (n, n, n)
    return np.asarray(rho, dtype=np.float64).reshape(shape), np.asarray(u, dtype=np.float64).reshape((len(u),) + shape), shape
