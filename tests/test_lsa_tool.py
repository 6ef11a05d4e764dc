"""Host logic of the stability-analysis tool (`paper_1505_06900_amd.lsa`), on the CPU.

The tool measures Lambda on the GPU; here it is handed the oracle's complex-step Lambda instead
and its host side is checked against independent facts:
* its velocity table is the library's documented population order, the one the oracle uses;
* with Lambda = identity (pure streaming) the eigenvalues are exp(-i k.xi_j), so omega_j = k.xi_j;
* the paper's stability statements (Sec. 3.6, tau = 0.5001, D2Q9 order 4: stable at u_x = 0.2,
  unstable at 0.248; order 2 unstable along k_y = 0 at 0.2) hold through its eigenvalue path;
* at small k the three least damped modes follow its Navier-Stokes relations (Sec. 3.6):
  Im omega = -nu k^2 for shear and, with the BGK bulk viscosity, for sound; Re omega_+- = +-c_s k
  + k.u and Re omega_s = k.u;
* the onset search brackets the root of a synthetic growth function and handles the stable and
  already-unstable ends;
* the five-point difference weights differentiate quartics exactly.
"""
import numpy as np
import pytest

from oracle import lattice as OL
from oracle import lsa as OLSA
from paper_1505_06900_amd import lsa


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
def test_velocity_table_is_the_documented_population_order(lat):
    c = lsa.velocity_set(lat)
    L = OL.lattice(lat)
    assert c.shape == (L.q, 3)
    np.testing.assert_array_equal(c[:, : L.D], L.c[:, : L.D])
    if lat != "D3Q19":
        cz = c[:, 2] if lat == "D3Q27" else 0
        assert (np.arange(L.q) == (c[:, 0] + 1) + 3 * (c[:, 1] + 1) + 9 * (cz + 1) * (lat == "D3Q27")).all()


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q27"])
def test_pure_streaming_has_omega_k_dot_xi(lat):
    q = lsa.velocity_set(lat).shape[0]
    k = np.array([[0.3, -1.1, 0.7], [2.0, 0.5, -0.4]])
    w = lsa.omega(lsa.amplification_eigenvalues(np.eye(q), lat, k))
    expect = k @ lsa.velocity_set(lat).T.astype(float)
    for r in range(k.shape[0]):
        # Re omega is defined modulo 2 pi: compare on the unit circle
        got = np.sort(np.angle(np.exp(1j * w[r].real)))
        ref = np.sort(np.angle(np.exp(1j * expect[r])))
        np.testing.assert_allclose(got, ref, atol=1e-12)
        np.testing.assert_allclose(w[r].imag, 0.0, atol=1e-12)


def _oracle_J(order, tau, u, lat="D2Q9"):
    return OLSA.jacobian(lat, order, tau, 1.0, u)


def test_paper_stability_statements_through_the_host_path():
    J02 = _oracle_J(4, 0.5001, [0.2, 0.0])
    J0248 = _oracle_J(4, 0.5001, [0.248, 0.0])
    g02 = lsa.max_growth("D2Q9", 4, 0.5001, [[0.2, 0.0]], nk=64, J=J02[None])[0]
    g0248 = lsa.max_growth("D2Q9", 4, 0.5001, [[0.248, 0.0]], nk=64, J=J0248[None])[0]
    assert g02 < 1e-10 and g0248 > 1e-6  # 1.37e-5 on this grid
    # agrees with the oracle's own k-grid evaluation
    assert g0248 == pytest.approx(OLSA.max_growth("D2Q9", 4, 0.5001, 1.0, np.array([0.248, 0.0]), nk=64), rel=1e-9)
    _, w = lsa.dispersion_kx("D2Q9", 2, 0.5001, [0.2, 0.0], nk=401, J=_oracle_J(2, 0.5001, [0.2, 0.0]))
    assert w.imag.max() > 1e-7
    kx, ky, m = lsa.dissipation_map("D2Q9", 4, 0.5001, [0.2, 0.0], nk=32, J=J02)
    assert m.shape == (32, 32) and kx[0] == -np.pi and m.max() < 1e-10


def test_small_k_modes_follow_navier_stokes():
    tau, u = 0.8, np.array([0.05, 0.0])
    nu = (tau - 0.5) / 3
    k = np.array([0.04, 0.0])
    w = lsa.modes("D2Q9", 4, tau, u, k, J=_oracle_J(4, tau, u))[:3]  # least damped: two sound, shear
    ns = lsa.navier_stokes(k, u, nu, 2)
    ref = np.array([ns["plus"], ns["minus"], ns["shear"]])
    got = w[np.argsort(-w.real)]
    ref = ref[np.argsort(-ref.real)]
    np.testing.assert_allclose(got.real, ref.real, rtol=1e-3)
    np.testing.assert_allclose(got.imag, ref.imag, rtol=2e-2)


def test_onset_search_on_a_synthetic_growth():
    root = 0.23456
    s = lsa.bracket_onset(lambda v: np.asarray(v) - root, 0.0, 0.6, tol_u=1e-5)
    assert root <= s <= root + 1e-5
    assert lsa.bracket_onset(lambda v: -np.ones_like(v), 0.0, 0.6) is None
    assert lsa.bracket_onset(lambda v: np.ones_like(v), 0.1, 0.6) == 0.1


def test_five_point_weights_differentiate_quartics_exactly():
    h = 0.1
    p = np.polynomial.Polynomial([0.3, -1.2, 0.7, 2.5, -0.9])
    x0 = 0.37
    d = (8 * (p(x0 + h) - p(x0 - h)) - (p(x0 + 2 * h) - p(x0 - 2 * h))) / (12 * h)
    assert d == pytest.approx(p.deriv()(x0), abs=1e-12)
    assert lsa._STENCIL == (1.0, -1.0, 2.0, -2.0)
