"""Oracle of the learned-closure data pipeline (D2Q9), FP64.

Test infrastructure only (see the package docstring).

The closure is not part of the paper.  It corrects the off-equilibrium
coefficient a1^(2) of a coarse run (Sec. 2: P^(1) = a1^(2)) before the
recursion of Sec. 3.1 rebuilds the higher orders.  Definitions used here and
by the GPU path:

coarse-graining (factor F, acoustic scaling: dx_c = dt_c = F dx_f, so
velocities and stresses keep their lattice-unit values):
    rho_c = box(rho_f),  j_c = box(rho_f u_f),  u_c = j_c / rho_c,
    T     = box(rho_f u_f u_f) - rho_c u_c u_c          (sub-filter stress),
    A_c*  = [box((1 - 1/(2 tau_f)) A_f) + T] / (1 - 1/(2 tau_c)),
where box averages the F x F fine nodes of a coarse node and A_f is the
pre-collision a1^(2) of the fine run.  (1 - 1/(2 tau)) A is the viscous part of
the momentum flux of the scheme (average of the pre- and post-collision
a1^(2)), so A_c* is the coarse a1^(2) whose momentum flux equals the filtered
fine flux.

features of a coarse node at the next step, from a stored post-collision
state g (the same definition is used by the fused inference kernel):
    9 pulled pre-collision deviations f_i(x) - w_i rho0,  f_i(x) = g_i(x - xi_i);
    then, for the 3 x 3 neighbours x + (dx, dy), dy = -1, 0, 1 (outer),
    dx = -1, 0, 1 (inner): rho - rho0, u_x, u_y of g at that neighbour.
The plain scheme's a1^(2) at x is that of the pulled populations.
"""
from __future__ import annotations

import numpy as np

from . import rr
from .lattice import lattice

PAIRS2D = [(0, 0), (0, 1), (1, 1)]  # packed order xx, xy, yy


def box(a, F):
    """Mean over F x F blocks of the last two axes."""
    *lead, ny, nx = a.shape
    return a.reshape(*lead, ny // F, F, nx // F, F).mean(axis=(-3, -1))


def coarse_target(rho_f, u_f, A_f, tau_f, tau_c, F):
    """(rho_c, u_c, A_c* packed (3, ...)) from fine fields rho_f (ny, nx), u_f (2, ny, nx),
    A_f packed (3, ny, nx)."""
    rho_c = box(rho_f, F)
    j_c = box(rho_f * u_f, F)
    u_c = j_c / rho_c
    visc = box((1.0 - 0.5 / tau_f) * A_f, F)
    T = np.stack([box(rho_f * u_f[a] * u_f[b], F) - rho_c * u_c[a] * u_c[b] for (a, b) in PAIRS2D])
    return rho_c, u_c, (visc + T) / (1.0 - 0.5 / tau_c)


def features(g, rho0=1.0):
    """Features (n_nodes, 36) and plain a1^(2) packed (n_nodes, 3) of the step after state g.

    g: post-collision populations (9, 1, ny, nx) in canonical D2Q9 order."""
    L = lattice("D2Q9")
    f = rr.stream(L, g)  # pulled pre-collision populations at every node
    rho_f, u_f, Pi = rr.moments(L, f)
    A = rr.offeq_second(L, rho_f, u_f, Pi)
    rho_g, u_g, _ = rr.moments(L, g)
    ny, nx = g.shape[-2:]
    cols = [f[i, 0] - L.w[i] * rho0 for i in range(9)]
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            # value at x + (dx, dy): roll by (-dy, -dx)
            sh = lambda a: np.roll(a[0], shift=(-dy, -dx), axis=(0, 1))
            cols += [sh(rho_g) - rho0, sh(u_g[0]), sh(u_g[1])]
    X = np.stack([c.reshape(-1) for c in cols], axis=1)
    Ap = np.stack([A[a, b, 0].reshape(-1) for (a, b) in PAIRS2D], axis=1)
    return X, Ap
