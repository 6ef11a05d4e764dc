"""Pins of the closure oracle (MLP and coarse-graining), which has no counterpart in the paper.

* GELU: gelu(x) - gelu(-x) = x, gelu(0) = 0, gelu'(0) = 1/2, gelu' = finite differences;
* BF16 rounding: nearest-even on hand-made halfway cases;
* backward pass: exact (unrounded) gradients equal central finite differences of the loss;
* Adam: the first update is -lr g / (|g| + eps) (closed form);
* coarse-graining: constants are preserved, a uniform flow has no sub-filter stress, a linear
  shear u_x = a y has T_xx = a^2 (F^2 - 1)/12, the target of a uniform a1^(2) scales by
  (1 - 1/(2 tau_f)) / (1 - 1/(2 tau_c));
* features: equal a brute-force node-by-node gather on a small grid.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closure as OC
from oracle import lattice as OL
from oracle import mlp as OM
from oracle import rr


def test_gelu_identities_and_derivative():
    x = np.linspace(-5, 5, 101)
    np.testing.assert_allclose(OM.gelu(x) - OM.gelu(-x), x, atol=1e-14)
    assert OM.gelu(np.array([0.0]))[0] == 0.0
    assert OM.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-15)
    h = 1e-6
    fd = (OM.gelu(x + h) - OM.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(OM.gelu_grad(x), fd, atol=1e-8)
    # large |z|: gelu -> relu
    assert OM.gelu(np.array([8.0]))[0] == pytest.approx(8.0, abs=1e-12)
    assert OM.gelu(np.array([-8.0]))[0] == pytest.approx(0.0, abs=1e-12)


def test_bf16_round_to_nearest_even():
    u = 2.0**-7  # BF16 spacing just above 1
    cases = [(1.0, 1.0), (1 + u / 2, 1.0), (1 + 1.5 * u, 1 + 2 * u), (1 + 0.51 * u, 1 + u),
             (-(1 + 1.5 * u), -(1 + 2 * u)), (3.0, 3.0), (0.1, 0.10009765625), (0.0, 0.0)]
    for a, b in cases:
        assert OM.bf16(np.array([a]))[0] == b, (a, b)


def test_backward_equals_finite_differences():
    rng = np.random.default_rng(0)
    p = OM.init_params(1).astype(np.float64) + 0.05 * rng.standard_normal(OM.NPARAM)
    x = rng.standard_normal((8, OM.NIN))
    t = rng.standard_normal((8, OM.NOUT))
    _, g = OM.backward(p, x, t, rounding=False)
    h = 1e-6
    idx = rng.choice(OM.NPARAM, size=60, replace=False)
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (OM.loss(OM.forward(p + e, x, False)[0], t) - OM.loss(OM.forward(p - e, x, False)[0], t)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-10), k


def test_rounded_network_is_close_to_exact():
    rng = np.random.default_rng(2)
    p = OM.init_params(3).astype(np.float64)
    x = rng.standard_normal((16, OM.NIN))
    y1, _ = OM.forward(p, x, True)
    y0, _ = OM.forward(p, x, False)
    assert np.abs(y1 - y0).max() < 0.05 * np.abs(y0).max()
    assert np.abs(y1 - y0).max() > 0  # rounding points are active


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = OM.adam(p, np.zeros(50), np.zeros(50), g, 1, lr=1e-3, eps=1e-8)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_coarse_graining_closed_forms():
    F, n = 4, 16
    rho = np.full((n, n), 1.03)
    u = np.zeros((2, n, n))
    u[0] = 0.07
    u[1] = -0.02
    A = np.zeros((3, n, n))
    rc, uc, Ac = OC.coarse_target(rho, u, A, 0.6, 0.52, F)
    np.testing.assert_allclose(rc, 1.03)
    np.testing.assert_allclose(uc[0], 0.07)
    np.testing.assert_allclose(Ac, 0.0, atol=1e-17)
    # linear shear: T_xx = a^2 (F^2 - 1)/12, T_xy = T_yy = 0
    a = 1e-3
    y = np.arange(n, dtype=float)
    u = np.zeros((2, n, n))
    u[0] = a * y[:, None]
    rho = np.ones((n, n))
    _, _, Ac = OC.coarse_target(rho, u, np.zeros((3, n, n)), 0.6, 0.6, F)
    np.testing.assert_allclose(Ac[0] * (1 - 0.5 / 0.6), a * a * (F * F - 1) / 12, rtol=1e-10)
    np.testing.assert_allclose(Ac[1:], 0.0, atol=1e-18)
    # uniform a1^(2) at rest scales with the viscous factors
    A = np.ones((3, n, n)) * np.array([2e-4, -1e-4, 3e-4])[:, None, None]
    _, _, Ac = OC.coarse_target(np.ones((n, n)), np.zeros((2, n, n)), A, 0.6, 0.52, F)
    np.testing.assert_allclose(Ac, A[:, ::F, ::F] * (1 - 0.5 / 0.6) / (1 - 0.5 / 0.52), rtol=1e-12)


def test_features_match_brute_force_gather():
    L = OL.lattice("D2Q9")
    ny, nx = 5, 7
    rho, u, pi1 = (1.0 + W.smooth_random(1, (1, ny, nx), 0.02, 1)[0],
                   W.smooth_random(2, (1, ny, nx), 0.05, 2), W.smooth_random(3, (1, ny, nx), 1e-3, 3))
    f = rr.init_populations(L, 4, rho, u, rr.pi1_from_components(L, pi1))
    g = rr.collide(L, 4, 0.7, f) + W.noise(f.shape, 1e-4, 4)
    X, Ap = OC.features(g)
    assert X.shape == (ny * nx, 36) and Ap.shape == (ny * nx, 3)
    for y in range(ny):
        for x in range(nx):
            row = X[y * nx + x]
            pulled = np.array([g[i, 0, (y - L.c[i, 1]) % ny, (x - L.c[i, 0]) % nx] for i in range(9)])
            np.testing.assert_allclose(row[:9], pulled - L.w, atol=1e-15)
            k = 9
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    gg = g[:, 0, (y + dy) % ny, (x + dx) % nx]
                    r = gg.sum()
                    jx = (gg * L.c[:, 0]).sum()
                    jy = (gg * L.c[:, 1]).sum()
                    np.testing.assert_allclose(row[k:k + 3], [r - 1.0, jx / r, jy / r], atol=1e-15)
                    k += 3
            # plain a1^(2) of the pulled populations
            r = pulled.sum()
            ux, uy = (pulled * L.c[:, 0]).sum() / r, (pulled * L.c[:, 1]).sum() / r
            axx = (pulled * L.c[:, 0] ** 2).sum() - r / 3 - r * ux * ux
            axy = (pulled * L.c[:, 0] * L.c[:, 1]).sum() - r * ux * uy
            ayy = (pulled * L.c[:, 1] ** 2).sum() - r / 3 - r * uy * uy
            np.testing.assert_allclose(Ap[y * nx + x], [axx, axy, ayy], atol=1e-15)


def test_flux_label_factor_from_the_steady_response():
    """Iterate the a1^(2) recursion A <- A_s + omega (A + D) of a constant correction D and check that
    the steady flux, half the sum of the pre- and post-collision moments, carries omega D/(1 - omega);
    D = flux_label_factor(tau) * T then carries exactly T."""
    for tau in (0.508868, 0.6, 0.9):
        om = 1 - 1 / tau
        A_s, T = 3e-4, 2e-6
        D = OC.flux_label_factor(tau) * T
        A = 0.0
        for _ in range(5000):
            A = A_s + om * (A + D)
        flux_with = 0.5 * (A + om * (A + D))
        A0 = 0.0
        for _ in range(5000):
            A0 = A_s + om * A0
        flux_without = 0.5 * (A0 + om * A0)
        assert flux_with - flux_without == pytest.approx(T, rel=1e-9)
        assert flux_without == pytest.approx((1 - 0.5 / tau) * A0, rel=1e-12)
