"""Oracle of resting no-slip walls for the regularised scheme, FP64.

Test infrastructure only (see the package docstring).

The paper's Dirichlet boundary (Sec. 3.7, "Boundary conditions"): at a
boundary node the velocity u_bc is imposed, rho is obtained from the
symmetries of the lattice, f0 follows from (rho, u_bc), the off-equilibrium
stress P^(1) is obtained from the lattice symmetries, f1 is built from it
(Eq. fone_d2q9 / fone_d3q27, which for u_bc = 0 reduces to the second-order
term), and every population of the node is replaced by f0 + f1.  The collision
that follows is the ordinary regularised one.

Walls here: u_bc = 0 on the first and last node of each walled axis (the
walls lie on the nodes).  Reading of "the symmetries of the lattice" (the
paper defers to the literature for it): after streaming, a population of a
wall node whose source node lies outside the box is unknown;
  * an unknown population whose opposite population is known takes the
    opposite's off-equilibrium part: f_i - w_i rho = f_opp - w_opp rho (with
    w_i = w_opp this is f_i = f_opp);
  * an unknown population whose opposite is unknown too (edges and corners)
    is taken at equilibrium, f_i = w_i rho;
  * rho is the zeroth moment of the completed set, which fixes it:
    rho (1 - sum_buried w_i) = sum_known f_i + sum_bounced f_opp.
P^(1) = a1^(2) is then the second moment of f - w rho of the completed set
(u_bc = 0), and the node's populations become f0(rho, 0) + f1(0, a1^(2)).
"""
from __future__ import annotations

import numpy as np

from . import rr
from .lattice import lattice


def _lat(lat):
    return lattice(lat) if isinstance(lat, str) else lat


def opposite(L):
    """Index of -xi_i for every population i."""
    c = L.c
    idx = np.array([int(np.where((c == -c[i]).all(axis=1))[0][0]) for i in range(L.q)])
    return idx


def unknown_mask(lat, shape, walls):
    """(q, nz, ny, nx) mask of the populations whose source node x - xi_i lies outside the box.

    walls = (x, y, z) booleans: that axis is bounded by walls on its first and last node."""
    L = _lat(lat)
    nz, ny, nx = shape
    coords = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    z, y, x = coords
    unk = np.zeros((L.q,) + tuple(shape), dtype=bool)
    for i, (cx, cy, cz) in enumerate(L.c):
        out = np.zeros(shape, dtype=bool)
        for walled, pos, c, n in ((walls[0], x, cx, nx), (walls[1], y, cy, ny), (walls[2], z, cz, nz)):
            if walled:
                src = pos - c
                out |= (src < 0) | (src >= n)
        unk[i] = out
    return unk


def regularize_walls(lat, N, f, walls, n1=None):
    """Replace the populations of every wall node of a streamed state f (q, nz, ny, nx) by the
    regularised no-slip populations f0(rho, 0) + f1(0, a1^(2)) (f1 at order n1, default
    ``rr.f1_order(lat, N)``)."""
    L = _lat(lat)
    unk = unknown_mask(L, f.shape[1:], walls)
    wall = unk.any(axis=0)
    if not wall.any():
        return f
    opp = opposite(L)
    known = ~unk
    bounced = unk & known[opp]
    buried = unk & unk[opp]
    w = L.w.reshape((-1,) + (1,) * (f.ndim - 1))
    s = np.where(known, f, 0.0).sum(axis=0) + np.where(bounced, f[opp], 0.0).sum(axis=0)
    wb = np.where(buried, w, 0.0).sum(axis=0)
    rho = s / (1.0 - wb)
    fneq = np.where(known, f - w * rho, 0.0) + np.where(bounced, f[opp] - w[opp] * rho, 0.0)
    c = L.c.astype(float)
    A = np.einsum("ia,ib,i...->ab...", c, c, fneq)  # a1^(2) with u = 0
    if L.D == 2:
        A[2, :] = 0.0
        A[:, 2] = 0.0
    zero_u = np.zeros((L.D,) + rho.shape)
    n1 = rr.f1_order(L, N) if n1 is None else n1
    freg = rr.reconstruct(L, N, rr.a0_coefficients(L, N, rho, zero_u)) + rr.reconstruct(
        L, n1, rr.a1_coefficients(L, n1, A, zero_u))
    return np.where(wall[None], freg, f)


def step_walls(lat, N, tau, f, walls, n1=None):
    """One time step on pre-collision populations with resting walls: collide, stream, regularise
    the wall nodes."""
    L = _lat(lat)
    return regularize_walls(L, N, rr.stream(L, rr.collide(L, N, tau, f, n1)), walls, n1)


def run_walls(lat, N, tau, rho, u, steps, walls, pi1=None, n1=None):
    """Evolve from fields (u = 0 expected on the wall nodes) for ``steps`` steps; returns
    pre-collision populations."""
    L = _lat(lat)
    f = rr.init_populations(L, N, rho, u, pi1, n1)
    for _ in range(steps):
        f = step_walls(L, N, tau, f, walls, n1)
    return f


def one_sided_derivative(a, axis, walled):
    """d a / d axis by second-order central differences; on a walled axis the first and last
    node use the second-order one-sided formulas (-3 a0 + 4 a1 - a2)/2 and (3 an - 4 an-1 + an-2)/2."""
    d = 0.5 * (np.roll(a, -1, axis=axis) - np.roll(a, 1, axis=axis))
    if walled:
        a0 = np.take(a, 0, axis=axis)
        a1 = np.take(a, 1, axis=axis)
        a2 = np.take(a, 2, axis=axis)
        n = a.shape[axis]
        b0 = np.take(a, n - 1, axis=axis)
        b1 = np.take(a, n - 2, axis=axis)
        b2 = np.take(a, n - 3, axis=axis)
        idx0 = [slice(None)] * a.ndim
        idx0[axis] = 0
        idxn = [slice(None)] * a.ndim
        idxn[axis] = n - 1
        d[tuple(idx0)] = 0.5 * (-3.0 * a0 + 4.0 * a1 - a2)
        d[tuple(idxn)] = 0.5 * (3.0 * b0 - 4.0 * b1 + b2)
    return d


def trapezoid_mean(a, walls):
    """Mean of a (nz, ny, nx) field over the box by the trapezoid rule on walled axes.

    A walled axis of n nodes has its walls on the first and last node: the box spans n - 1
    cells along it and those two nodes weigh 1/2.  A periodic axis of n nodes spans n cells of
    weight 1 (the plain mean)."""
    X, Y, Z = 2, 1, 0
    w = np.ones_like(a)
    vol = 1.0
    for k, ax in ((0, X), (1, Y), (2, Z)):
        n = a.shape[ax]
        if k < len(walls) and walls[k]:
            wt = np.ones(n)
            wt[0] = wt[-1] = 0.5
            shape = [1, 1, 1]
            shape[ax] = n
            w = w * wt.reshape(shape)
            vol *= n - 1
        else:
            vol *= n
    return float(np.sum(w * a) / vol)


def enstrophy_walls(u, walls):
    """Enstrophy of Sec. 4.1 (half the integral of |omega|^2) over the box, divided by its
    volume: one-sided differences on the walls, trapezoid rule on walled axes (u: (D, nz, ny, nx))."""
    X, Y, Z = 2, 1, 0
    dd = lambda a, ax, k: one_sided_derivative(a, ax, walls[k])
    if u.shape[0] == 2:
        w = dd(u[1], X, 0) - dd(u[0], Y, 1)
        return trapezoid_mean(0.5 * w * w, walls)
    ux, uy, uz = u
    wx = dd(uz, Y, 1) - dd(uy, Z, 2)
    wy = dd(ux, Z, 2) - dd(uz, X, 0)
    wz = dd(uy, X, 0) - dd(ux, Y, 1)
    return trapezoid_mean(0.5 * (wx * wx + wy * wy + wz * wz), walls)
