"""Dipole-wall collision (Sec. 4.1): a self-propelled dipole in the box [-1, 1]^2 with no-slip
walls, Re = 2500, run with the library's wall step; the two enstrophy peaks are compared with the
reference values the paper quotes (3313 and 1418).

Orchestration only: the steps, the enstrophy integral (lb_enstrophy, trapezoid rule between the
walls) and the kinetic energy (lb_reduce) run in liblbrr.so.  Only the largest local speed of the
constant-Mach runs (their Mach number) is taken with torch from the velocity field lb_moments
returns.

Scaling (a reading of Sec. 4.1, where the printed rule U_lb = 0.01 N/125 contradicts the stated
constant viscosity): N nodes per unit length (walls on the first and last of 2N + 1 nodes),
U_lb = 0.01 * 125 / N, so nu_lb = U_lb N / Re = 5e-4 and tau = 0.5015 at every resolution, and the
Mach number falls as 1/N (the compressibility reduction the paper invokes).  Physical time
t = steps * U_lb / N.  Initial state: rho = 1, u from Eqs. dipole1 / dipole2 (the paper sets up its
initial condition by an iterative procedure of its reference, not given; here the populations
start at the regularised equilibrium).
"""
from __future__ import annotations

import time

import numpy as np

from . import LB_ERR_UNSTABLE, LBError, Simulation

RE = 2500.0
REFERENCE_PEAKS = (3313.0, 1418.0)


def lattice_parameters(n_unit, u_lb=None):
    """(U_lb, nu, tau) at N nodes per unit length: U_lb = 0.01 * 125 / N unless given (the
    constant-Mach runs of Sec. 4.1 keep U_lb fixed and let the viscosity follow Re)."""
    if u_lb is None:
        u_lb = 0.01 * 125.0 / n_unit
    nu = u_lb * n_unit / RE
    return u_lb, nu, 3.0 * nu + 0.5


def _torch():
    import torch

    return torch


def enstrophy_integral(sim, u_lb):
    """<Omega> = 1/2 int omega^2 dx dy over the box in the paper's units, from lb_enstrophy: half
    the trapezoid-rule integral of the lattice vorticity squared (second-order differences,
    one-sided on the walls) over the (m - 1)^2 cells between the wall nodes, divided by their
    number; omega is per lattice step, so the paper's vorticity is omega / U_lb in its units."""
    m = sim.nx
    return sim.enstrophy() * (m - 1) ** 2 / (u_lb * u_lb)


def kinetic_energy(sim, u_lb):
    """1/2 int rho |u|^2 dx dy in the paper's units from lb_reduce (the wall nodes carry u = 0,
    so the sum over the nodes is the trapezoid rule)."""
    n_unit = (sim.nx - 1) // 2
    return sim.reduce()[4] / (u_lb * u_lb * n_unit * n_unit)


def run(n_unit, t_end=1.0, dt_sample=0.002, storage="fp64", order=4, log=None, u_lb=None, track_mach=None):
    """Evolve the dipole to t_end; returns dict(times, enstrophy, energy, peaks, errors, ...).

    u_lb: lattice velocity unit (default 0.01 * 125 / N, the constant-viscosity series); a fixed
    value gives the constant-Mach series (U_lb = 0.032: the Ma 0.7 runs of Sec. 4.1).
    log: optional callable, given a progress line every 100 samples.
    track_mach: also record the largest |u| of every sample (default: with a fixed u_lb)."""
    import workloads as W

    torch = _torch()
    if track_mach is None:
        track_mach = u_lb is not None
    u_lb, nu, tau = lattice_parameters(n_unit, u_lb)
    u_phys, _ = W.dipole(n_unit)
    m = 2 * n_unit + 1
    sim = Simulation("D2Q9", (1, m, m), tau, order, storage=storage)
    sim.set_walls(x=True, y=True)
    sim.init_fields(np.ones((1, m, m)), u_lb * u_phys)
    steps_per_unit = n_unit / u_lb
    every = max(1, int(round(dt_sample * steps_per_unit)))
    total = int(round(t_end * steps_per_unit))
    times, ens, ke = [], [], []
    umax = 0.0
    t0 = time.perf_counter()
    k = 0
    while True:
        times.append(k / steps_per_unit)
        try:
            e_k, k_k = enstrophy_integral(sim, u_lb), kinetic_energy(sim, u_lb)
        except LBError as e:  # the run lost its finite state
            if e.code != LB_ERR_UNSTABLE:
                raise
            e_k = k_k = float("nan")
        ens.append(e_k)
        ke.append(k_k)
        if not np.isfinite(e_k):
            break
        if track_mach:  # the largest local speed, for the Mach number of the constant-Mach runs
            _, v = sim.moments(torch.float64)
            umax = max(umax, float(torch.sqrt(v[0] ** 2 + v[1] ** 2).max()))
        if log is not None and len(times) % 100 == 0:
            log(f"dipole N={n_unit} {storage}: t = {times[-1]:.3f}, enstrophy {ens[-1]:.1f}")
        if k >= total:
            break
        n = min(every, total - k)
        sim.step(n)
        k += n
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    times, ens = np.array(times), np.array(ens)
    peaks = []
    for lo, hi in ((0.2, 0.5), (0.5, 0.9)):
        sel = (times >= lo) & (times <= hi)
        if sel.any():
            i = int(np.argmax(np.where(sel, ens, -np.inf)))
            peaks.append((float(times[i]), float(ens[i])))
    errors = [abs(p[1] - r) / r for p, r in zip(peaks, REFERENCE_PEAKS)]
    return {"n_unit": n_unit, "nodes": m * m, "u_lb": u_lb, "tau": tau, "steps": k, "storage": storage,
            "umax": umax,
            "times": times, "enstrophy": ens, "energy": np.array(ke), "peaks": peaks, "errors": errors,
            "wall_s": wall, "glups": m * m * k / wall / 1e9}
