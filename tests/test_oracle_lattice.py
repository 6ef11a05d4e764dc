"""Pins of the oracle's lattice tables against the mathematics and the paper.

The velocity sets must be Gauss--Hermite quadratures exact to 5th order
(Sec. 3.2); the Hermite basis must be orthogonal on D2Q9 / D3Q27 with the
normalisations that reproduce every printed prefactor of Eqs. fzero_d2q9,
fone_d2q9, fzero_d3q27 and fone_d3q27; D3Q19 at second order must reduce to
the textbook second-order equilibrium.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import lattice as Lm
from oracle import rr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gauss_moment(n, cs2):
    return 0.0 if n % 2 else cs2 ** (n // 2) * math.prod(range(n - 1, 0, -2))


def test_d1q3_is_three_point_rule():
    xi, w, cs2 = Lm.d1q3()
    assert list(xi) == [-1, 0, 1]
    np.testing.assert_allclose(w, [1 / 6, 2 / 3, 1 / 6], rtol=1e-14)
    assert cs2 == pytest.approx(1 / 3, rel=1e-14)
    assert Lm.CS2 == pytest.approx(cs2, rel=1e-14)


def test_mach_numbers_printed_in_paper_fix_cs():
    # Sec. 3.6: u = 0.2 <-> Ma 0.346 and u = 0.248 <-> Ma 0.43 => c_s = 1/sqrt(3)
    cs = math.sqrt(Lm.CS2)
    assert 0.2 / cs == pytest.approx(0.346, abs=5e-4)
    assert 0.248 / cs == pytest.approx(0.43, abs=5e-3)


@pytest.mark.parametrize("name", Lm.LATTICES)
def test_quadrature_exact_to_fifth_order(name):
    L = Lm.lattice(name)
    c = L.c
    for p, q, s in itertools.product(range(6), repeat=3):
        if p + q + s > 5 or (L.D == 2 and s):
            continue
        num = np.sum(L.w * c[:, 0] ** p * c[:, 1] ** q * c[:, 2] ** s)
        ref = gauss_moment(p, L.cs2) * gauss_moment(q, L.cs2) * gauss_moment(s, L.cs2)
        assert num == pytest.approx(ref, abs=1e-15), (name, p, q, s)


def test_d3q19_weights_solve_exactly():
    vel, w, resid = Lm.d3q19_weights()
    assert resid < 1e-15
    assert len(vel) == 19
    cls = np.sum(vel**2, axis=1)
    np.testing.assert_allclose(w[cls == 0], 1 / 3, rtol=1e-14)
    np.testing.assert_allclose(w[cls == 1], 1 / 18, rtol=1e-14)
    np.testing.assert_allclose(w[cls == 2], 1 / 36, rtol=1e-14)


@pytest.mark.parametrize("name", Lm.LATTICES)
def test_opposites(name):
    L = Lm.lattice(name)
    for i in range(L.q):
        assert tuple(L.c[L.opposite(i)]) == tuple(-L.c[i])


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_gram_is_diagonal_with_closed_form_norms(name):
    L = Lm.lattice(name)
    N = Lm.MAX_ORDER[name]
    G = L.gram(N)
    np.testing.assert_allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-15)
    for r, (a, b, c) in enumerate(L.basis):
        n = a + b + c
        ref = math.factorial(a) * math.factorial(b) * math.factorial(c) * L.cs2**n
        assert G[r, r] == pytest.approx(ref, rel=1e-13)
    assert np.linalg.matrix_rank(L.H) == L.q  # complete basis of the population space


def test_d3q19_basis_rank_and_couplings():
    L = Lm.lattice("D3Q19")
    assert np.linalg.matrix_rank(L.H) == 19
    G = L.gram(4)
    idx = {k: r for r, k in enumerate(L.basis)}
    # third-order pairs that share the odd axis are coupled on D3Q19 (not on D3Q27)
    assert G[idx[(1, 2, 0)], idx[(1, 0, 2)]] == pytest.approx(-1 / 27, abs=1e-15)
    assert G[idx[(1, 2, 0)], idx[(1, 2, 0)]] == pytest.approx(2 / 27, abs=1e-15)
    assert G[idx[(0, 0, 2)], idx[(2, 2, 0)]] == pytest.approx(-1 / 27, abs=1e-15)
    assert G[idx[(2, 2, 0)], idx[(2, 0, 2)]] == pytest.approx(-1 / 81, abs=1e-15)
    # orders 0-2 remain orthogonal (quadrature exact to 5th order)
    low = [r for r, k in enumerate(L.basis) if sum(k) <= 2]
    Gl = G[np.ix_(low, low)]
    np.testing.assert_allclose(Gl - np.diag(np.diag(Gl)), 0.0, atol=1e-15)


def _prefactors():
    rows = []
    with open(os.path.join(GOLDEN, "hermite_prefactors.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            lat, term, num, den, n = line.split()
            rows.append((lat, term, int(num), int(den), int(n)))
    return rows


@pytest.mark.parametrize("row", _prefactors(), ids=lambda r: f"{r[0]}-{r[1]}")
def test_printed_prefactors(row):
    """The printed prefactor of each Hermite term equals 1/N_k of the oracle's basis."""
    lat, term, num, den, n = row
    L = Lm.lattice(lat)
    k = (0, 0, 0) if term == "-" else tuple(term.count(ax) for ax in "xyz")
    assert sum(k) == n
    r = L.basis.index(k)
    printed = num / (den * L.cs2**n)
    assert 1.0 / L.norms[r] == pytest.approx(printed, rel=1e-13)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_second_order_equilibrium_is_textbook(name):
    """At N = 2, f0 = w rho (1 + xi.u/cs2 + (xi.u)^2/(2 cs4) - u.u/(2 cs2)) (Eq. feq_2, Sec. 3.8.1)."""
    L = Lm.lattice(name)
    rng = np.random.default_rng(3)
    rho = 1 + 0.05 * rng.standard_normal(7)
    u = 0.1 * rng.standard_normal((L.D, 7))
    f0 = rr.init_populations(L, 2, rho, u)
    c = L.c[:, : L.D].astype(float)
    cu = c @ u
    ref = L.w[:, None] * rho * (1 + cu / L.cs2 + cu**2 / (2 * L.cs2**2) - np.sum(u * u, 0) / (2 * L.cs2))
    np.testing.assert_allclose(f0, ref, rtol=1e-14, atol=1e-16)
