"""Oracle recursive-regularised collision and streaming, FP64.

Test infrastructure only (see the package docstring).

The scheme, in the paper's order:

1. macroscopic moments rho, rho u and the second moment Pi of the
   (pre-collision) populations -- Sec. 2, Eqs. def_rho, def_j, def_p
   (written here with raw second moments sum_i xi_i xi_i f_i);
2. equilibrium Hermite coefficients a0^(n) = rho u...u -- Sec. 2,
   Eqs. a^0_0 .. a^3_0 and the recursion a0^(n) = a0^(n-1) u of Sec. 3.1;
3. second-order off-equilibrium coefficient a1^(2) = P^(1), obtained as
   the projection of f - f0 on H^(2) (Sec. 2; Sec. 3.5 says this is done as in
   the earlier regularised model): a1^(2) = Pi - rho c_s^2 I - rho u u;
4. higher-order a1^(n) by the recursion of Sec. 3.1, Eq. rel_a1 (proved in
   App. A), with the discrete O(Ma^(n+1)) terms of App. B dropped as the paper
   does;
5. reconstruction of f0 and f1 on the lattice's Hermite basis truncated at
   order N (Eqs. fzero_d2q9 / fone_d2q9, fzero_d3q27 / fone_d3q27), written
   as the Gram projection f = W H^T G^-1 a (identical to the printed formulas
   for D2Q9 / D3Q27, whose Gram matrix is diagonal); on D3Q19 f1 stops at
   order 3 (``f1_order``);
6. post-collision populations f0 + (1 - 1/tau) f1 -- Sec. 3.5, Eq.
   discr_bgk_reg, with tau the shifted relaxation time of Sec. 3.4
   (Eq. full_discr_bgk), so nu = c_s^2 (tau - 1/2);
7. streaming f_i(x + xi_i, t + 1) = post-collision f_i(x, t), periodic.

Shapes: populations (q, ...) with any trailing node shape; for ``stream`` the
trailing shape must be (nz, ny, nx).  ``u`` is (D, ...); the second-order
tensors (Pi, a1^(2)) are (3, 3, ...) full symmetric arrays.
"""
from __future__ import annotations

import numpy as np

from .lattice import Lattice, lattice, tuple_of

CS2 = 1.0 / 3.0


def _lat(lat):
    return lattice(lat) if isinstance(lat, str) else lat


def moments(lat, f):
    """rho, u (D, ...), Pi (3, 3, ...) = sum_i xi_i xi_i f_i."""
    L = _lat(lat)
    c = L.c.astype(float)
    rho = f.sum(axis=0)
    j = np.tensordot(c.T, f, axes=(1, 0))      # (3, ...)
    Pi = np.einsum("ia,ib,i...->ab...", c, c, f)
    u = j[: L.D] / rho
    return rho, u, Pi


def _u3(u):
    """Pad a (D, ...) velocity to three components (u_z = 0 in 2D)."""
    if u.shape[0] == 3:
        return u
    return np.concatenate([u, np.zeros((3 - u.shape[0],) + u.shape[1:], dtype=u.dtype)])


def offeq_second(lat, rho, u, Pi):
    """a1^(2) = Pi - rho c_s^2 I - rho u u (Sec. 2, P^(1) = a1^(2))."""
    u3 = _u3(u)
    A = Pi - rho * np.einsum("a...,b...->ab...", u3, u3)
    for a in range(3):
        A[a, a] = A[a, a] - rho * CS2
    L = _lat(lat)
    if L.D == 2:  # no z direction on a 2D lattice
        A[2, :] = 0.0
        A[:, 2] = 0.0
    return A


def a0_coefficients(lat, N, rho, u):
    """Equilibrium Hermite coefficients a0_k = rho u_x^a u_y^b u_z^c, |k| <= N, shape (K_N, ...)."""
    L = _lat(lat)
    u3 = _u3(u)
    out = []
    for r in L.kept(N):
        k = L.basis[r]
        # recursion a0^(n) = a0^(n-1) u_alpha_n applied along the index tuple
        val = rho
        for alpha in tuple_of(k):
            val = val * u3[alpha]
        out.append(val)
    return np.stack(out)


def a1_tuple(A, u3, t, memo):
    """a1 for index tuple t by Eq. rel_a1 (Sec. 3.1), discrete error terms dropped (App. B).

    a1(a_1..a_n) = a1(a_1..a_{n-1}) u_{a_n}
                   + sum over the n-1 cyclic shifts of (a_1..a_{n-1}) of
                     u_{a_1} ... u_{a_{n-2}} a1^(2)_{a_{n-1} a_n},
    i.e. every a_j (j < n) is paired once with a_n in a1^(2), the other
    n-2 indices of the first n-1 going into velocity factors.
    """
    if t in memo:
        return memo[t]
    n = len(t)
    if n < 2:
        val = np.zeros_like(u3[0])          # a1^(0) = a1^(1) = 0 by construction
    elif n == 2:
        val = A[t[0], t[1]]
    else:
        head, last = t[:-1], t[-1]
        val = a1_tuple(A, u3, head, memo) * u3[last]
        for j in range(n - 1):
            term = A[head[j], last]
            for l in range(n - 1):
                if l != j:
                    term = term * u3[head[l]]
            val = val + term
    memo[t] = val
    return val


def a1_coefficients(lat, N, A, u):
    """Off-equilibrium Hermite coefficients a1_k for |k| <= N, shape (K_N, ...)."""
    L = _lat(lat)
    u3 = _u3(u)
    memo = {}
    return np.stack([a1_tuple(A, u3, tuple_of(L.basis[r]), memo) * np.ones_like(u3[0])
                     for r in L.kept(N)])


def reconstruct(lat, N, a):
    """Populations whose projections on the kept Hermite polynomials equal ``a`` (Eq. hermite_eq)."""
    L = _lat(lat)
    R = L.recon_matrix(N)
    return np.tensordot(R, a, axes=(1, 0))


def f1_order(lat, N):
    """Hermite order of the off-equilibrium part f1 when f0 is truncated at order N.

    N on D2Q9 and D3Q27.  D3Q19 has no complete Hermite basis (Sec. 3.2) and the paper
    leaves its generalisation open (Sec. 5); on it f1 stops at order 3 while f0 keeps
    order N.  The alternative, an f1 at order 4 carrying the recursion's fourth-order
    coefficients through the Gram projection, makes the linearised collision grow at
    rest for tau close to 1/2 (the analysis of Sec. 3.6, ``test_oracle_lsa``); with f1
    at order 3 the rest state is stable at every tau."""
    L = _lat(lat)
    return min(N, 3) if L.name == "D3Q19" else N


def collide(lat, N, tau, f, n1=None):
    """Post-collision populations f0 + (1 - 1/tau) f1 (Eq. discr_bgk_reg), per node.

    f0 is reconstructed at order N, f1 at order n1 (default ``f1_order(lat, N)``)."""
    n1 = f1_order(lat, N) if n1 is None else n1
    rho, u, Pi = moments(lat, f)
    A = offeq_second(lat, rho, u, Pi)
    f0 = reconstruct(lat, N, a0_coefficients(lat, N, rho, u))
    f1 = reconstruct(lat, n1, a1_coefficients(lat, n1, A, u))
    return f0 + (1.0 - 1.0 / tau) * f1


def stream(lat, f):
    """Periodic streaming: out_i(x + xi_i) = f_i(x); f shape (q, nz, ny, nx)."""
    L = _lat(lat)
    out = np.empty_like(f)
    for i, (cx, cy, cz) in enumerate(L.c):
        out[i] = np.roll(f[i], shift=(int(cz), int(cy), int(cx)), axis=(0, 1, 2))
    return out


def step(lat, N, tau, f, n1=None):
    """One time step on pre-collision populations (Eq. discr_bgk_reg as printed: collide, then stream)."""
    return stream(lat, collide(lat, N, tau, f, n1))


def step_post(lat, N, tau, g, n1=None):
    """One time step on post-collision populations: stream, then collide.

    A state stored after the collision (g = collide(f)) advances by
    g(t+1) = collide(stream(g(t))); the moments rho, u of g(t) and f(t) agree
    because the collision conserves them.
    """
    return collide(lat, N, tau, stream(lat, g), n1)


def init_populations(lat, N, rho, u, pi1=None, n1=None):
    """Pre-collision populations f0^(N)(rho, u) [+ f1^(n1)(u, a1^(2) = pi1)] at t = 0.

    ``pi1`` is a full (3, 3, ...) symmetric tensor or None.  Higher-order
    off-equilibrium coefficients come from the recursion, as in the collision;
    n1 defaults to ``f1_order(lat, N)``.
    """
    f = reconstruct(lat, N, a0_coefficients(lat, N, rho, u))
    if pi1 is not None:
        n1 = f1_order(lat, N) if n1 is None else n1
        f = f + reconstruct(lat, n1, a1_coefficients(lat, n1, pi1, u))
    return f


def pi1_from_components(lat, comps):
    """Full (3,3,...) tensor from packed components: 2D (xx, xy, yy), 3D (xx, xy, xz, yy, yz, zz)."""
    L = _lat(lat)
    shape = comps.shape[1:]
    A = np.zeros((3, 3) + shape)
    pairs = [(0, 0), (0, 1), (1, 1)] if L.D == 2 else [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for n, (a, b) in enumerate(pairs):
        A[a, b] = comps[n]
        A[b, a] = comps[n]
    return A


def pi1_components(lat, A):
    """Packed components of a full (3,3,...) tensor (inverse of ``pi1_from_components``)."""
    L = _lat(lat)
    pairs = [(0, 0), (0, 1), (1, 1)] if L.D == 2 else [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    return np.stack([A[a, b] for (a, b) in pairs])


def run(lat, N, tau, rho, u, steps, pi1=None, n1=None):
    """Evolve from fields for ``steps`` steps (push form); returns pre-collision populations."""
    f = init_populations(lat, N, rho, u, pi1, n1)
    for _ in range(steps):
        f = step(lat, N, tau, f, n1)
    return f
