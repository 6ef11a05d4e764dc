"""Von Neumann linear stability analysis of the library's own scheme (Sec. 3.6).

The update is linearised about a uniform state f = f0(rho, u): a perturbation f' obeys
f'(x + xi_i, t + 1) = sum_j Lambda_ij f'_j(x, t) with Lambda_ij = d Omega_i / d f_j (Eq. lin1), and a
plane wave exp(i k.x) turns this into the q x q amplification matrix A^-1 Lambda,
A^-1 = diag(exp(-i k.xi_j)) (Eq. lin2).  Its eigenvalues lambda_j give the dispersion and
dissipation omega_j = i log lambda_j: Re omega_j = -arg lambda_j, Im omega_j = ln |lambda_j|, and a
mode grows when Im omega_j > 0.

Lambda is measured from the library's FP64 step itself, so the analysis covers exactly the
collision the kernels compute.  A box of cells of 5^D nodes is set to uniform states.  In each
cell, population j of the centre node gets one perturbation of the stored state: +h, -h, +2h
or -2h.  One step (pull, then collide) brings it to the node xi_j away.  That node then holds
Omega(f + s h e_j), and every population it pulls comes from inside the cell.  The five-point
difference [8 (Omega(+h) - Omega(-h)) - (Omega(+2h) - Omega(-2h))] / (12 h) gives column j of
Lambda, with an error of O(h^4).  Many uniform states share one box and one step.  The
eigenvalues come from numpy's LAPACK binding; the paper says it used a linear algebra
package.

Functions: ``jacobians`` (Lambda for a batch of states), ``modes`` (omega over a set of
wavevectors), ``dispersion_kx`` (omega along k_x), ``dissipation_map`` (max_j Im omega over a
k-grid, the maps of Sec. 3.6), ``max_growth`` and ``stability_threshold`` (the smallest speed
along a direction with a growing mode), and ``navier_stokes`` (the Navier-Stokes
dispersion-dissipation relations the paper compares with).  ``python -m
paper_1505_06900_amd.lsa {kx,map,threshold} ...`` writes them to an .npz file and prints a
one-line JSON summary.
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from . import DIM, Q, Simulation

CELL = 5  # nodes per cell edge: the output node and everything it pulls stay inside
_STENCIL = (1.0, -1.0, 2.0, -2.0)  # perturbations in units of h


def velocity_set(lattice):
    """Discrete velocities (q, 3) in the library's population order: i = (cx+1) + 3(cy+1) + 9(cz+1)
    for D2Q9 (cz = 0) and D3Q27; D3Q19 keeps that order without the 8 corners."""
    r = (-1, 0, 1)
    if lattice == "D2Q9":
        return np.array([(cx, cy, 0) for cy in r for cx in r], dtype=np.int64)
    full = [(cx, cy, cz) for cz in r for cy in r for cx in r]
    if lattice == "D3Q27":
        return np.array(full, dtype=np.int64)
    if lattice == "D3Q19":
        return np.array([c for c in full if sum(abs(v) for v in c) < 3], dtype=np.int64)
    raise ValueError(f"unknown lattice {lattice!r}")


def _torch():
    import torch

    return torch


def jacobians(lattice, order, tau, velocities, rho=1.0, h=3e-4):
    """Lambda = dOmega/df (nb, q, q) at f0(rho, u) for each row u of ``velocities`` (nb, D),
    measured from one FP64 step of the library (see the module docstring)."""
    torch = _torch()
    D, q = DIM[lattice], Q[lattice]
    vel = np.atleast_2d(np.asarray(velocities, dtype=np.float64))
    if vel.shape[1] != D:
        raise ValueError(f"velocities must have {D} components")
    nb = vel.shape[0]
    c = velocity_set(lattice)
    ns = len(_STENCIL)
    ncell = nb * q * ns
    ncx = min(ncell, 64)
    ncy = -(-ncell // ncx)
    nz = CELL if D == 3 else 1
    shape = (nz, CELL * ncy, CELL * ncx)

    # uniform state of each cell: cell k belongs to state k // (q * ns); padding cells take state 0
    cell_of_y = np.arange(shape[1]) // CELL
    cell_of_x = np.arange(shape[2]) // CELL
    cell = cell_of_y[:, None] * ncx + cell_of_x[None, :]
    state = np.where(cell < ncell, cell // (q * ns), 0)
    u2 = np.moveaxis(vel[state], -1, 0)  # (D, ny, nx)
    u = np.broadcast_to(u2[:, None], (D,) + shape).copy()
    sim = Simulation(lattice, shape, tau, order, storage="fp64", rho0=1.0)
    try:
        sim.init_fields(np.full(shape, float(rho)), u)
        f = sim.get_populations()
        k = np.arange(ncell)
        b, j, s = k // (q * ns), (k // ns) % q, k % ns
        zc = np.full(ncell, nz // 2)
        yc = CELL * (k // ncx) + CELL // 2
        xc = CELL * (k % ncx) + CELL // 2
        dev = f.device
        idx = lambda a: torch.as_tensor(a, device=dev)
        amp = torch.as_tensor(np.asarray(_STENCIL)[s] * h, device=dev, dtype=torch.float64)
        f[idx(j), idx(zc), idx(yc), idx(xc)] += amp
        sim.set_populations(f)
        sim.step(1)
        g = sim.get_populations()
        cj = c[j]
        out = g[:, idx(zc + cj[:, 2]), idx(yc + cj[:, 1]), idx(xc + cj[:, 0])]  # (q, ncell)
        out = out.cpu().numpy().T.reshape(nb, q, ns, q)  # [state, column j, stencil point, row i]
    finally:
        sim.close()
    d1 = out[:, :, 0, :] - out[:, :, 1, :]
    d2 = out[:, :, 2, :] - out[:, :, 3, :]
    return np.swapaxes((8.0 * d1 - d2) / (12.0 * h), 1, 2)  # [state, row i, column j]


def _k_points(k):
    k = np.asarray(k, dtype=np.float64)
    if k.shape[-1] == 2:
        k = np.concatenate([k, np.zeros(k.shape[:-1] + (1,))], axis=-1)
    return k


def amplification_eigenvalues(J, lattice, k):
    """Eigenvalues (..., q) of A^-1 Lambda = diag(exp(-i k.xi)) J at wavevectors k (..., 2 or 3)."""
    c = velocity_set(lattice).astype(np.float64)
    k = _k_points(k)
    phase = np.exp(-1j * (k @ c.T))  # (..., q)
    return np.linalg.eigvals(phase[..., :, None] * J)


def omega(lam):
    """omega = i log lambda (Re: dispersion, Im: dissipation; Im > 0 grows; a zero eigenvalue
    gives Im omega = -inf)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return 1j * np.log(lam)


def _log_modulus(lam):
    with np.errstate(divide="ignore"):
        return np.log(np.abs(lam))


def modes(lattice, order, tau, u, k, rho=1.0, J=None):
    """omega_j(k) (..., q) for the uniform state (rho, u); modes sorted by Im omega, least damped first."""
    if J is None:
        J = jacobians(lattice, order, tau, [u], rho)[0]
    w = omega(amplification_eigenvalues(J, lattice, k))
    order_ = np.argsort(-w.imag, axis=-1)
    return np.take_along_axis(w, order_, axis=-1)


def k_grid(nk, D=2):
    """The grid [-pi, pi)^D with nk points per axis, as (nk, ..., nk, D) wavevectors."""
    k1 = -np.pi + 2.0 * np.pi * np.arange(nk) / nk
    return np.stack(np.meshgrid(*([k1] * D), indexing="ij"), axis=-1)


def dispersion_kx(lattice, order, tau, u, nk=129, rho=1.0, J=None):
    """(kx in [0, pi], omega (nk, q)) along k_y = k_z = 0."""
    kx = np.linspace(0.0, np.pi, nk)
    k = np.zeros((nk, 3))
    k[:, 0] = kx
    return kx, modes(lattice, order, tau, u, k, rho, J)


def dissipation_map(lattice, order, tau, u, nk=64, kz=0.0, rho=1.0, J=None):
    """(kx, ky, max_j Im omega_j (nk, nk)) over [-pi, pi)^2 at the given k_z."""
    if J is None:
        J = jacobians(lattice, order, tau, [u], rho)[0]
    k2 = k_grid(nk, 2)
    k = np.concatenate([k2, np.full(k2.shape[:-1] + (1,), float(kz))], axis=-1)
    grow = _log_modulus(amplification_eigenvalues(J, lattice, k)).max(axis=-1)
    k1 = k2[:, 0, 0]
    return k1, k1.copy(), grow


def max_growth(lattice, order, tau, velocities, nk=64, rho=1.0, J=None):
    """max over the k-grid [-pi, pi)^D (nk per axis; nk <= 24 is advisable in 3D) and the modes of
    Im omega, for each row of ``velocities``."""
    D = DIM[lattice]
    if J is None:
        J = jacobians(lattice, order, tau, velocities, rho)
    k = k_grid(nk, D).reshape(-1, D)
    out = np.empty(J.shape[0])
    for b in range(J.shape[0]):
        g = -np.inf
        for chunk in np.array_split(k, max(1, k.shape[0] // 8192)):
            g = max(g, float(_log_modulus(amplification_eigenvalues(J[b], lattice, chunk)).max()))
        out[b] = g
    return out


def bracket_onset(growth, lo, hi, tol_u=1e-4, per_round=33, tol_growth=1e-8):
    """Smallest speed s in [lo, hi] with growth(s) > tol_growth, to within tol_u, assuming that the
    unstable speeds form an interval [s*, hi].  growth takes an array of speeds and returns one
    value per speed.  Returns None when hi is stable and lo when lo is already unstable."""
    s = np.linspace(lo, hi, per_round)
    g = np.asarray(growth(s))
    if not (g > tol_growth).any():
        return None
    i = int(np.argmax(g > tol_growth))
    if i == 0:
        return float(lo)
    a, b = s[i - 1], s[i]
    while b - a > tol_u:
        s = np.linspace(a, b, per_round)
        g = np.asarray(growth(s))
        i = int(np.argmax(g > tol_growth)) if (g > tol_growth).any() else len(s) - 1
        a, b = s[max(i - 1, 0)], s[i]
    return float(b)


def stability_threshold(lattice, order, tau, direction=(1.0, 0.0), nk=64, lo=0.0, hi=0.6, tol_u=1e-4,
                        rho=1.0, tol_growth=1e-8):
    """Smallest |u| along ``direction`` at which a mode grows on the nk-point k-grid (None if
    stable up to hi)."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)

    def growth(speeds):
        vel = np.asarray(speeds)[:, None] * d[None, :]
        return max_growth(lattice, order, tau, vel, nk, rho)

    return bracket_onset(growth, lo, hi, tol_u, tol_growth=tol_growth)


def navier_stokes(k, u, nu, D, eta=None):
    """Dispersion-dissipation relations of the linearised Navier-Stokes equations (Sec. 3.6):
    acoustic omega_+-, shear omega_s; eta (bulk viscosity) defaults to 2 nu / D, the BGK value.
    k (..., D), u (D,); returns a dict of complex arrays."""
    k = np.asarray(k, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    eta = 2.0 * nu / D if eta is None else eta
    kn = np.linalg.norm(k, axis=-1)
    ku = k @ u
    cs = math.sqrt(1.0 / 3.0)
    damp_ac = -kn**2 * 0.5 * ((2.0 * D - 2.0) / D * nu + eta)
    return {"plus": kn * cs + ku + 1j * damp_ac, "minus": -kn * cs + ku + 1j * damp_ac,
            "shear": ku - 1j * kn**2 * nu}


def main(argv=None):
    p = argparse.ArgumentParser(prog="python -m paper_1505_06900_amd.lsa", description=__doc__.split("\n\n")[0])
    p.add_argument("what", choices=["kx", "map", "threshold"])
    p.add_argument("--lattice", default="D2Q9", choices=sorted(Q))
    p.add_argument("--order", type=int, default=4)
    p.add_argument("--tau", type=float, default=0.5001)
    p.add_argument("--u", type=float, nargs="+", default=[0.2, 0.0], help="velocity of the uniform state")
    p.add_argument("--direction", type=float, nargs="+", default=None, help="threshold search direction")
    p.add_argument("--nk", type=int, default=64)
    p.add_argument("--kz", type=float, default=0.0)
    p.add_argument("--out", default=None, help=".npz file for the arrays")
    a = p.parse_args(argv)
    D = DIM[a.lattice]
    u = np.zeros(D)
    u[: min(D, len(a.u))] = a.u[:D]
    summary = {"what": a.what, "lattice": a.lattice, "order": a.order, "tau": a.tau, "u": u.tolist(), "nk": a.nk}
    arrays = {}
    if a.what == "kx":
        kx, w = dispersion_kx(a.lattice, a.order, a.tau, u, a.nk)
        arrays = {"kx": kx, "re_omega": w.real, "im_omega": w.imag}
        summary["max_im_omega"] = float(w.imag.max())
    elif a.what == "map":
        kx, ky, g = dissipation_map(a.lattice, a.order, a.tau, u, a.nk, a.kz)
        arrays = {"kx": kx, "ky": ky, "max_im_omega": g}
        summary["max_im_omega"] = float(g.max())
        summary["unstable_fraction"] = float((g > 1e-8).mean())
    else:
        d = np.zeros(D)
        src = a.direction if a.direction is not None else [1.0]
        d[: min(D, len(src))] = src[:D]
        s = stability_threshold(a.lattice, a.order, a.tau, d, a.nk)
        summary["direction"] = d.tolist()
        summary["threshold_speed"] = s
        summary["threshold_mach"] = None if s is None else s / math.sqrt(1.0 / 3.0)
    if a.out:
        np.savez(a.out, **arrays)
        summary["out"] = a.out
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
