"""Pins of the oracle's collision against the paper and against brute force.

* the recursion (Sec. 3.1, Eq. rel_a1) against the paper's explicit formulas
  of App. B (2D and 3D, orders 3-6, discrete error terms dropped as App. B
  says) and against the pair-sum closed form it implies;
* reconstruction against a dense linear solve and projection identities;
* the equilibrium as a fixed point, conservation of mass and momentum
  (Sec. 2: the collision conserves the first two moments);
* the recursion against the directly projected third/fourth-order moments of
  plain BGK runs (Sec. 3.3, Eq. rel_a1_lowma: agreement up to O(Ma^(n+1)));
* a z-invariant 3D run against the 2D run (the marginal of the 3D scheme).
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import lattice as Lm
from oracle import rr

RNG = np.random.default_rng(1234)


def rand_state(D, n=11, amp_u=0.15, amp_a=0.02, seed=0):
    rng = np.random.default_rng(seed)
    u = amp_u * rng.standard_normal((3, n))
    if D == 2:
        u[2] = 0.0
    B = amp_a * rng.standard_normal((3, 3, n))
    A = 0.5 * (B + B.transpose(1, 0, 2))
    if D == 2:
        A[2, :] = 0.0
        A[:, 2] = 0.0
    return u, A


def app_b_2d(u, A):
    """App. B, two dimensions (a1^(3)_xxy in a1^(4)_xxyy read with the subscript 1 the text omits)."""
    ux, uy = u[0], u[1]
    xyy = ux * A[1, 1] + 2 * uy * A[0, 1]
    xxy = 2 * ux * A[0, 1] + uy * A[0, 0]
    xxyy = uy * xxy + ux**2 * A[1, 1] + 2 * ux * uy * A[0, 1]
    return {(1, 2, 0): xyy, (2, 1, 0): xxy, (2, 2, 0): xxyy}


def app_b_3d(u, A):
    """App. B, three dimensions, orders 3 to 6."""
    ux, uy, uz = u
    xx, yy, zz, xy, xz, yz = A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]
    r = {}
    r[(2, 1, 0)] = 2 * ux * xy + uy * xx
    r[(2, 0, 1)] = 2 * ux * xz + uz * xx
    r[(1, 2, 0)] = ux * yy + 2 * uy * xy
    r[(1, 0, 2)] = ux * zz + 2 * uz * xz
    r[(0, 1, 2)] = uy * zz + 2 * uz * yz
    r[(0, 2, 1)] = 2 * uy * yz + uz * yy
    r[(1, 1, 1)] = ux * yz + uy * xz + uz * xy
    r[(2, 2, 0)] = ux**2 * yy + 2 * ux * uy * xy + uy * r[(2, 1, 0)]
    r[(2, 0, 2)] = ux**2 * zz + 2 * ux * uz * xz + uz * r[(2, 0, 1)]
    r[(0, 2, 2)] = uy**2 * zz + 2 * uy * uz * yz + uz * r[(0, 2, 1)]
    r[(1, 1, 2)] = ux * uy * zz + ux * uz * yz + uy * uz * xz + uz * r[(1, 1, 1)]
    r[(1, 2, 1)] = 2 * ux * uy * yz + uy**2 * xz + uz * r[(1, 2, 0)]
    r[(2, 1, 1)] = ux**2 * yz + 2 * ux * uy * xz + uz * r[(2, 1, 0)]
    r[(2, 1, 2)] = ux**2 * uy * zz + ux**2 * uz * yz + 2 * ux * uy * uz * xz + uz * r[(2, 1, 1)]
    r[(2, 2, 1)] = 2 * ux**2 * uy * yz + 2 * ux * uy**2 * xz + uz * r[(2, 2, 0)]
    r[(1, 2, 2)] = ux * uy**2 * zz + 2 * ux * uy * uz * yz + uy**2 * uz * xz + uz * r[(1, 2, 1)]
    r[(2, 2, 2)] = ux**2 * uy**2 * zz + 2 * ux**2 * uy * uz * yz + 2 * ux * uy**2 * uz * xz + uz * r[(2, 2, 1)]
    return r


def pair_sum(u, A, k):
    """Closed form implied by Eq. rel_a1: sum over index pairs of a1^(2) times the other velocities."""
    t = Lm.tuple_of(k)
    n = len(t)
    out = np.zeros_like(u[0])
    for j, l in itertools.combinations(range(n), 2):
        term = A[t[j], t[l]]
        for m in range(n):
            if m not in (j, l):
                term = term * u[t[m]]
        out = out + term
    return out


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_recursion_matches_appendix_b(name):
    L = Lm.lattice(name)
    u, A = rand_state(L.D)
    N = Lm.MAX_ORDER[name]
    a1 = rr.a1_coefficients(L, N, A, u[: L.D])
    ref = app_b_2d(u, A) if L.D == 2 else app_b_3d(u, A)
    kept = [L.basis[r] for r in L.kept(N)]
    for k, val in ref.items():
        np.testing.assert_allclose(a1[kept.index(k)], val, rtol=1e-13, atol=1e-16, err_msg=str(k))
    # second order returns a1^(2) itself, orders 0 and 1 vanish
    for r, k in enumerate(kept):
        if sum(k) < 2:
            assert np.all(a1[r] == 0)
        elif sum(k) == 2:
            t = Lm.tuple_of(k)
            np.testing.assert_array_equal(a1[r], A[t[0], t[1]])


@pytest.mark.parametrize("name", Lm.LATTICES)
def test_recursion_matches_pair_sum(name):
    L = Lm.lattice(name)
    u, A = rand_state(L.D, seed=5)
    N = Lm.MAX_ORDER[name]
    a1 = rr.a1_coefficients(L, N, A, u[: L.D])
    for r, idx in enumerate(L.kept(N)):
        k = L.basis[idx]
        if sum(k) >= 2:
            np.testing.assert_allclose(a1[r], pair_sum(u, A, k), rtol=1e-13, atol=1e-17)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_projection_reconstruction_identity(name):
    """On a complete orthogonal basis, f -> Hermite moments -> f is the identity."""
    L = Lm.lattice(name)
    f = RNG.uniform(0.0, 1.0, size=(L.q, 6))
    a = L.H @ f
    np.testing.assert_allclose(rr.reconstruct(L, Lm.MAX_ORDER[name], a), f, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("name,N", [(n, N) for n in Lm.LATTICES for N in range(2, Lm.MAX_ORDER[n] + 1)])
def test_collision_projects_back_to_coefficients(name, N):
    """Projecting f_out on every H_k kept by f1 returns a0_k + (1-1/tau) a1_k, and f_out is the
    sum of the two minimum-norm (W^-1 metric) solutions of the moment constraints, f0 for a0 at
    order N and f1 for a1 at order n1 (n1 = N, or 3 on D3Q19), by dense solves."""
    L = Lm.lattice(name)
    tau = 0.73
    n1 = rr.f1_order(L, N)
    rho = 1 + 0.03 * RNG.standard_normal(5)
    u = 0.1 * RNG.standard_normal((L.D, 5))
    A = rr.pi1_from_components(L, 0.01 * RNG.standard_normal((3 if L.D == 2 else 6, 5)))
    f = rr.init_populations(L, N, rho, u, A)
    g = rr.collide(L, N, tau, f)
    a0 = rr.a0_coefficients(L, N, rho, u)
    a1 = rr.a1_coefficients(L, n1, A, u)
    H0, H1 = L.H[L.kept(N)], L.H[L.kept(n1)]
    a0_low = a0[[L.kept(N).index(r) for r in L.kept(n1)]]
    np.testing.assert_allclose(H1 @ g, a0_low + (1 - 1 / tau) * a1, rtol=1e-12, atol=1e-15)
    W = np.diag(L.w)
    for n in range(5):
        f0 = W @ H0.T @ np.linalg.solve(H0 @ W @ H0.T, a0[:, n])
        f1 = W @ H1.T @ np.linalg.solve(H1 @ W @ H1.T, a1[:, n])
        np.testing.assert_allclose(g[:, n], f0 + (1 - 1 / tau) * f1, rtol=1e-12, atol=1e-15)
    if len(L.kept(N)) == L.q and n1 == N:  # complete basis: the constraints alone fix f
        target = a0 + (1 - 1 / tau) * a1
        for n in range(5):
            np.testing.assert_allclose(g[:, n], np.linalg.solve(H0, target[:, n]), rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("name,N", [(n, N) for n in Lm.LATTICES for N in range(2, Lm.MAX_ORDER[n] + 1)])
def test_equilibrium_is_fixed_point(name, N):
    L = Lm.lattice(name)
    rho = 1 + 0.05 * RNG.standard_normal(9)
    u = 0.2 * RNG.standard_normal((L.D, 9))
    f0 = rr.init_populations(L, N, rho, u)
    _, _, Pi = rr.moments(L, f0)
    rho_m, u_m, _ = rr.moments(L, f0)
    np.testing.assert_allclose(rho_m, rho, rtol=1e-15)
    np.testing.assert_allclose(u_m, u, rtol=1e-13, atol=1e-16)
    A = rr.offeq_second(L, rho_m, u_m, Pi)
    np.testing.assert_allclose(A, 0.0, atol=1e-15)
    np.testing.assert_allclose(rr.collide(L, N, 0.61, f0), f0, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("name", Lm.LATTICES)
def test_uniform_flow_is_fixed_point_of_full_step(name):
    L = Lm.lattice(name)
    N = Lm.MAX_ORDER[name]
    shape = (1, 5, 6) if L.D == 2 else (4, 5, 6)
    rho = np.full(shape, 1.02)
    u = np.zeros((L.D,) + shape)
    u[0] = 0.13
    u[1] = -0.07
    f = rr.init_populations(L, N, rho, u)
    g = rr.step(L, N, 0.55, f)
    np.testing.assert_allclose(g, f, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("name,N", [(n, N) for n in Lm.LATTICES for N in range(2, Lm.MAX_ORDER[n] + 1)])
def test_conservation(name, N):
    L = Lm.lattice(name)
    shape = (1, 8, 8) if L.D == 2 else (6, 6, 6)
    rng = np.random.default_rng(7)
    f = rr.init_populations(L, N, np.ones(shape), np.zeros((L.D,) + shape))
    f = f * (1 + 0.05 * rng.standard_normal(f.shape))  # arbitrary non-equilibrium start
    rho0, u0, _ = rr.moments(L, f)
    g = rr.collide(L, N, 0.8, f)
    rho1, u1, _ = rr.moments(L, g)
    np.testing.assert_allclose(rho1, rho0, rtol=1e-14)
    np.testing.assert_allclose(rho1 * u1, rho0 * u0, atol=1e-15)
    M0 = rho0.sum()
    P0 = (rho0 * u0).sum(axis=(1, 2, 3))
    for _ in range(30 if L.D == 3 else 200):
        f = rr.step(L, N, 0.8, f)
    rho2, u2, _ = rr.moments(L, f)
    assert abs(rho2.sum() - M0) / M0 < 1e-13
    np.testing.assert_allclose((rho2 * u2).sum(axis=(1, 2, 3)), P0, atol=1e-12)


def _bgk_run(u0, n, tau, steps):
    """Plain BGK (f -= (f - f0)/tau, f0 at full order 4) on the 2D TGV, push streaming.

    Used only to check the recursion against moments that the BGK dynamics
    produces by itself (Sec. 3.3).
    """
    L = Lm.lattice("D2Q9")
    rho, u = W.tgv2d(n, u0)
    f = rr.init_populations(L, 4, rho, u)
    for _ in range(steps):
        r, v, _ = rr.moments(L, f)
        f0 = rr.init_populations(L, 4, r, v)
        f = rr.stream(L, f - (f - f0) / tau)
    return L, f


@pytest.mark.slow
def test_recursion_reproduces_projected_bgk_moments():
    """The recursion describes the 3rd/4th-order off-equilibrium moments a plain BGK flow develops.

    Sec. 3.1 derives Eq. rel_a1 from the first-order Chapman--Enskog solution
    of BGK, and Sec. 3.3 states that on the lattice it holds up to
    higher-order terms.  A BGK run (no regularisation) of the 2D TGV at fixed
    Mach number is measured after its initial transient: the projections of
    f - f0 on H_xxy, H_xyy, H_xxyy are compared with the recursion evaluated
    on the run's own a1^(2) and u.  The mismatch must fall steadily as the
    Knudsen number k*tau falls (N doubles) and be small at N = 128.
    """
    errs3, errs4 = [], []
    for n in (16, 32, 64, 128):
        L, f = _bgk_run(0.05, n, 0.55, 60)
        rho, u, Pi = rr.moments(L, f)
        A = rr.offeq_second(L, rho, u, Pi)
        f0 = rr.init_populations(L, 4, rho, u)
        proj = L.H @ (f - f0).reshape(L.q, -1)
        rec = rr.a1_coefficients(L, 4, A, u).reshape(len(L.kept(4)), -1)
        kept = [L.basis[r] for r in L.kept(4)]

        def rel(k):
            p = proj[L.basis.index(k)]
            return np.linalg.norm(p - rec[kept.index(k)]) / np.linalg.norm(p)

        errs3.append(max(rel((2, 1, 0)), rel((1, 2, 0))))
        errs4.append(rel((2, 2, 0)))
    assert all(a > 1.6 * b for a, b in zip(errs3, errs3[1:])), errs3
    assert all(a > 1.6 * b for a, b in zip(errs4, errs4[1:])), errs4
    assert errs3[-1] < 0.05 and errs4[-1] < 0.2


@pytest.mark.parametrize("lat3,N", [("D3Q27", 2), ("D3Q27", 3), ("D3Q27", 4), ("D3Q19", 4)])
def test_z_invariant_3d_run_marginalises_to_2d(lat3, N):
    """Summing a z-invariant 3D run over c_z gives the D2Q9 run at the same order.

    Exact for D3Q27 (tensor-product lattice, h_1 and h_2 have zero marginal) and
    for D3Q19 with f0 and f1 both at order 4 (the Gram solve restores the
    marginals: this pins the Gram projection of the fourth-order D3Q19 basis).  The
    D3Q19 model used elsewhere stops f1 at order 3 (rr.f1_order), and D3Q19 at
    order 2-3 does not marginalise exactly; those are not asserted.
    """
    n, nz = 8, 3
    rho, u = W.tgv2d(n, 0.06)
    pi = rr.pi1_from_components("D2Q9", W.smooth_random(3, (1, n, n), 2e-3, 11))
    f2 = rr.init_populations("D2Q9", N, rho, u, pi)
    rho3 = np.repeat(rho, nz, 0)
    u3 = np.concatenate([np.repeat(u, nz, 1), np.zeros((1, nz, n, n))])
    pi3 = np.zeros((3, 3, nz, n, n))
    pi3[:2, :2] = np.repeat(pi[:2, :2], nz, 2)
    f3 = rr.init_populations(lat3, N, rho3, u3, pi3, n1=N)
    for _ in range(6):
        f2 = rr.step("D2Q9", N, 0.7, f2)
        f3 = rr.step(lat3, N, 0.7, f3, n1=N)
    L3, L2 = Lm.lattice(lat3), Lm.lattice("D2Q9")
    F = np.zeros_like(f2)
    for i, c in enumerate(L3.c):
        j = [jj for jj, cc in enumerate(L2.c) if cc[0] == c[0] and cc[1] == c[1]][0]
        F[j] += f3[i][0:1]
    np.testing.assert_allclose(F, f2, rtol=1e-13, atol=1e-15)
