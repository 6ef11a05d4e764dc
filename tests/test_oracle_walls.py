"""Pins of the no-slip wall oracle (regularised Dirichlet boundary of Sec. 3.7, u_bc = 0).

* the unknown populations of a wall node are exactly those whose source lies outside the box
  (brute force on a small box), and population q-1-i is the opposite of i on every lattice;
* a fluid at rest in a closed box is a fixed point;
* channel flow (walls in y, periodic x): the first Dirichlet shear mode u_x = u0 sin(pi y/(ny-1))
  decays at nu (pi/(ny-1))^2 (closed form of the diffusion equation with u = 0 on the wall nodes),
  with second-order convergence;
* a z-invariant D3Q27 / D3Q19 box (walls in x and y) marginalises to the D2Q9 box;
* a dipole mirror-symmetric about the box's mid-line y = 0 stays so (the reflection
  (u_x, u_y)(x, -y) = (u_x, -u_y)(x, y) maps solutions to solutions);
* the one-sided wall derivative is exact on quadratics.
"""
import numpy as np
import pytest

import workloads as W
from oracle import lattice as OL
from oracle import rr
from oracle import walls as OW


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
def test_opposite_and_unknown_populations(lat):
    L = OL.lattice(lat)
    assert (OW.opposite(L) == L.q - 1 - np.arange(L.q)).all()
    shape = (3, 4, 5) if L.D == 3 else (1, 4, 5)
    walls = (True, True, L.D == 3)
    unk = OW.unknown_mask(L, shape, walls)
    nz, ny, nx = shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for i, (cx, cy, cz) in enumerate(L.c):
                    sx, sy, sz = x - cx, y - cy, z - cz
                    outside = not (0 <= sx < nx) or not (0 <= sy < ny) or (walls[2] and not (0 <= sz < nz))
                    assert unk[i, z, y, x] == outside


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
def test_rest_in_a_closed_box_is_a_fixed_point(lat):
    L = OL.lattice(lat)
    shape = (4, 5, 6) if L.D == 3 else (1, 7, 6)
    f = rr.init_populations(L, 4, np.full(shape, 1.02), np.zeros((L.D,) + shape))
    g = f
    for _ in range(5):
        g = OW.step_walls(L, 4, 0.7, g, (True, True, L.D == 3))
    np.testing.assert_allclose(g, f, atol=1e-15)


def channel_rate(ny, tau=0.8, nx=4):
    L = OL.lattice("D2Q9")
    nu = (tau - 0.5) / 3
    y = np.arange(ny)
    u = np.zeros((2, 1, ny, nx))
    u[0] = 1e-4 * np.sin(np.pi * y / (ny - 1))[None, :, None]
    f = rr.init_populations(L, 4, np.ones((1, ny, nx)), u)
    T = int(0.3 * (ny - 1) ** 2 / (nu * np.pi**2))
    amps = {}
    for t in range(T + 1):
        if t in (T // 3, T):
            amps[t] = rr.moments(L, f)[1][0, 0, (ny - 1) // 2, 0]
        f = OW.step_walls(L, 4, tau, f, (False, True, False))
    rate = -np.log(amps[T] / amps[T // 3]) / (T - T // 3)
    return rate / (nu * (np.pi / (ny - 1)) ** 2)


def test_channel_shear_mode_decays_at_the_dirichlet_rate():
    e17, e33 = abs(channel_rate(17) - 1), abs(channel_rate(33) - 1)
    assert e17 < 2e-3 and e33 < 5e-4
    assert 3.0 < e17 / e33 < 5.0  # second order in the wall spacing


@pytest.mark.parametrize("lat3", ["D3Q27", "D3Q19"])
def test_z_invariant_box_marginalises_to_d2q9(lat3):
    L2, L3 = OL.lattice("D2Q9"), OL.lattice(lat3)
    ny, nx, nz = 9, 11, 3
    rho = 1.0 + W.smooth_random(1, (1, ny, nx), 0.01, 3)[0]
    u2 = W.smooth_random(2, (1, ny, nx), 0.03, 4)
    u2[:, :, [0, -1], :] = 0.0
    u2[:, :, :, [0, -1]] = 0.0
    f2 = rr.init_populations(L2, 4, rho, u2)
    u3 = np.zeros((3, nz, ny, nx))
    u3[:2] = np.repeat(u2, nz, axis=1)
    # f1 at order 4 on both lattices: the Gram projection of the fourth-order D3Q19 basis
    # marginalises exactly (the default D3Q19 model stops f1 at order 3 and does not)
    f3 = rr.init_populations(L3, 4, np.repeat(rho, nz, axis=0), u3, n1=4)
    for _ in range(20):
        f2 = OW.step_walls(L2, 4, 0.7, f2, (True, True, False))
        f3 = OW.step_walls(L3, 4, 0.7, f3, (True, True, False), n1=4)
    m = np.zeros_like(f2)
    for i, c in enumerate(L3.c):
        j = int(np.where((L2.c[:, 0] == c[0]) & (L2.c[:, 1] == c[1]))[0][0])
        m[j] += f3[i, :1]
    np.testing.assert_allclose(m, f2, atol=1e-13)


def test_mirror_symmetric_flow_stays_symmetric():
    L = OL.lattice("D2Q9")
    n = 21
    y = np.arange(n) - (n - 1) / 2
    X, Y = np.meshgrid(y, y)
    g1 = np.exp(-(X**2 + (Y - 3) ** 2) / 10)
    g2 = np.exp(-(X**2 + (Y + 3) ** 2) / 10)
    u = np.stack([-0.03 * Y * g1 + 0.03 * Y * g2, 0.03 * X * g1 - 0.03 * X * g2])[:, None]
    u[:, :, [0, -1], :] = 0.0
    u[:, :, :, [0, -1]] = 0.0
    f = rr.init_populations(L, 4, np.ones((1, n, n)), u)
    for _ in range(100):
        f = OW.step_walls(L, 4, 0.6, f, (True, True, False))
    _, v, _ = rr.moments(L, f)
    scale = np.abs(v).max()
    assert np.abs(v[0] - v[0][:, ::-1, :]).max() <= 1e-12 * scale  # u_x even in y
    assert np.abs(v[1] + v[1][:, ::-1, :]).max() <= 1e-12 * scale  # u_y odd in y
    assert scale > 1e-3


def test_one_sided_derivative_is_exact_on_quadratics():
    x = np.arange(7, dtype=float)
    a = (2.0 + 0.5 * x - 0.25 * x * x)[None, None, :]
    d = OW.one_sided_derivative(a, 2, True)
    np.testing.assert_allclose(d[0, 0], 0.5 - 0.5 * x, atol=1e-14)


def test_walled_enstrophy_converges_at_second_order_to_the_integral():
    """Channel profile u_x = sin(pi y), y = j/(ny - 1) in [0, 1] between walls on the first and
    last node (periodic x): omega = -(pi/(ny - 1)) cos(pi y) per node, so half the integral of
    omega^2 over the box divided by its volume is pi^2 / (4 (ny - 1)^2).  One-sided wall
    differences and the trapezoid rule are both second order: the relative error falls about
    4x per halving of the spacing (a plain mean over the nodes would give first order, 2x)."""
    def err(ny):
        y = np.arange(ny) / (ny - 1)
        ux = np.sin(np.pi * y)[None, :, None] * np.ones((1, ny, 8))
        u = np.stack([ux, np.zeros_like(ux)])
        e = OW.enstrophy_walls(u, (False, True))
        return abs(e * 4 * (ny - 1) ** 2 / np.pi**2 - 1)

    e = [err(n) for n in (33, 65, 129)]
    assert e[2] < 1e-3
    for a, b in zip(e, e[1:]):
        assert 3.3 < a / b < 4.5


def test_trapezoid_mean_weights_and_volume():
    a = np.arange(3 * 4 * 5, dtype=float).reshape(3, 4, 5)
    assert OW.trapezoid_mean(a, (False, False, False)) == pytest.approx(a.mean(), rel=1e-15)
    # walled y: rows 0 and 3 weigh 1/2, three cells
    wy = np.array([0.5, 1, 1, 0.5])[None, :, None]
    assert OW.trapezoid_mean(a, (False, True, False)) == pytest.approx(float((a * wy).sum()) / (3 * 3 * 5), rel=1e-15)
    # constant field: the mean is the constant whatever the walls
    assert OW.trapezoid_mean(np.full((3, 4, 5), 2.5), (True, True, True)) == pytest.approx(2.5, rel=1e-15)
