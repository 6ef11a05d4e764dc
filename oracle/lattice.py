"""Oracle lattice tables: velocities, weights, Hermite basis, Gram matrices.

Test infrastructure only (see the package docstring).

Follows Sec. 3.2 ("Discretization of the microscopic velocity space"):
velocity space is discretised by a Gauss--Hermite quadrature; D2Q9 and D3Q27
are the tensor products of the three-point rule, whose 9 / 27 Hermite
polynomials span the whole population space, while D3Q19 does not carry a
complete Hermite basis.  The paper does not print the velocities or weights;
here they are *derived*:

* the 1D three-point rule is numpy's probabilists' Gauss--Hermite rule scaled
  so that its abscissae are the integers {-1, 0, 1}; this fixes c_s^2 = 1/3;
* D2Q9 / D3Q27 are its tensor products;
* D3Q19 weights (rest / face / edge classes) are the least-squares solution of
  the isotropy conditions of the Gaussian up to 4th order (the solution is
  exact; the residual is returned for the tests).

Hermite polynomials in lattice units (the c_s factors of Eqs. fzero_d2q9 /
fzero_d3q27): 1D h_n(xi) = c_s^n He_n(xi / c_s), multi-dimensional
H_k(xi) = h_a(xi_x) h_b(xi_y) h_c(xi_z) for k = (a, b, c), a, b, c <= 2.

Canonical velocity order (the paper is silent): i = (cx+1) + 3(cy+1) + 9(cz+1)
for D2Q9 (cz = 0) and D3Q27; D3Q19 keeps the D3Q27 order with the 8 corners
removed.  In all three the opposite of i is q-1-i.

D3Q19 basis (reading of the paper's open point, Sec. 3.2 and Sec. 5): keep the
tensor Hermite polynomials with at least one zero exponent (19 of them);
those with three non-zero exponents vanish (xyz) or alias lower ones on the
D3Q19 velocity set.  Because they are not orthogonal under the D3Q19 weights,
reconstruction uses the Gram solve ``f = W H^T G^-1 a`` (for D2Q9 / D3Q27 G is
diagonal and this is exactly the paper's expansion).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np
from numpy.polynomial import hermite_e

CS2 = 1.0 / 3.0  # fixed by the integer abscissae of the three-point rule (checked in the tests)

LATTICES = ("D2Q9", "D3Q19", "D3Q27")
MAX_ORDER = {"D2Q9": 4, "D3Q19": 4, "D3Q27": 6}


def d1q3():
    """Three-point Gauss--Hermite rule in lattice units.

    Returns (xi, w, cs2): integer abscissae sorted ascending, weights summing
    to one, and the squared lattice sound speed implied by the scaling.
    """
    x, wt = hermite_e.hermegauss(3)  # weight function exp(-x^2/2)
    order = np.argsort(x)
    x, wt = x[order], wt[order] / wt.sum()
    scale = x[-1]  # largest abscissa sqrt(3) becomes the unit lattice link
    xi = x / scale
    xi_int = np.rint(xi).astype(int)
    assert np.allclose(xi, xi_int, atol=1e-14)
    cs2 = 1.0 / scale**2  # unit-variance Gaussian rescaled by 1/scale
    return xi_int, wt, cs2


def _product_set(dim):
    """Tensor-product velocity set and weights in canonical order."""
    xi1, w1, _ = d1q3()
    vel, wts = [], []
    zr = range(3) if dim == 3 else range(1)
    for kz in zr:
        for ky in range(3):
            for kx in range(3):
                cz = xi1[kz] if dim == 3 else 0
                vel.append((xi1[kx], xi1[ky], cz))
                wts.append(w1[kx] * w1[ky] * (w1[kz] if dim == 3 else 1.0))
    return np.array(vel, dtype=int), np.array(wts)


def _gauss_moment(n, cs2):
    """E[X^n] for X ~ N(0, cs2): closed form cs^n (n-1)!! for even n, else 0."""
    if n % 2:
        return 0.0
    dbl = 1.0
    for m in range(n - 1, 0, -2):
        dbl *= m
    return cs2 ** (n // 2) * dbl


def d3q19_weights():
    """Weights of the D3Q19 set from the isotropy conditions.

    Unknowns: rest, face (|c|^2 = 1) and edge (|c|^2 = 2) weights.  Conditions:
    the set integrates 1, xi_x^2, xi_x^4 and xi_x^2 xi_y^2 like the Gaussian of
    variance c_s^2.  Returns (velocities, weights, residual norm).
    """
    vel27, _ = _product_set(3)
    keep = np.sum(vel27**2, axis=1) <= 2
    vel = vel27[keep]
    cls = np.sum(vel**2, axis=1)  # 0 rest, 1 face, 2 edge
    monomials = [(0, 0, 0), (2, 0, 0), (4, 0, 0), (2, 2, 0)]
    M = np.zeros((len(monomials), 3))
    rhs = np.zeros(len(monomials))
    for r, (p, q, s) in enumerate(monomials):
        vals = vel[:, 0] ** p * vel[:, 1] ** q * vel[:, 2] ** s
        for k in range(3):
            M[r, k] = vals[cls == k].sum()
        rhs[r] = _gauss_moment(p, CS2) * _gauss_moment(q, CS2) * _gauss_moment(s, CS2)
    sol, *_ = np.linalg.lstsq(M, rhs, rcond=None)
    resid = float(np.linalg.norm(M @ sol - rhs))
    return vel, sol[cls], resid


def hermite_1d(n, xi, cs2=CS2):
    """h_n(xi) = c_s^n He_n(xi/c_s) (probabilists' Hermite polynomial)."""
    cs = np.sqrt(cs2)
    coef = np.zeros(n + 1)
    coef[n] = 1.0
    return cs**n * hermite_e.hermeval(np.asarray(xi, dtype=float) / cs, coef)


def basis_indices(name):
    """Hermite multi-indices k = (a, b, c) carried by the lattice, sorted by order."""
    if name == "D2Q9":
        ks = [(a, b, 0) for b in range(3) for a in range(3)]
    elif name == "D3Q27":
        ks = [(a, b, c) for c in range(3) for b in range(3) for a in range(3)]
    elif name == "D3Q19":
        ks = [(a, b, c) for c in range(3) for b in range(3) for a in range(3)
              if min(a, b, c) == 0]
    else:
        raise ValueError(name)
    return sorted(ks, key=lambda k: (sum(k), k[::-1]))


@dataclass
class Lattice:
    name: str
    D: int
    c: np.ndarray          # (q, 3) integer velocities (cz = 0 in 2D)
    w: np.ndarray          # (q,)
    cs2: float
    basis: list            # all multi-indices the lattice carries
    H: np.ndarray          # (K, q) H_k(xi_i)
    norms: np.ndarray      # (K,) sum_i w_i H_k(xi_i)^2
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def q(self):
        return len(self.w)

    def opposite(self, i):
        return self.q - 1 - i

    def kept(self, N):
        """Indices (into ``basis``) of the multi-indices of order <= N."""
        return [r for r, k in enumerate(self.basis) if sum(k) <= N]

    def gram(self, N):
        sel = self.kept(N)
        Hn = self.H[sel]
        return Hn @ np.diag(self.w) @ Hn.T

    def recon_matrix(self, N):
        """R_N = W H_N^T G_N^-1, shape (q, K_N): populations from Hermite coefficients."""
        if N not in self._cache:
            sel = self.kept(N)
            Hn = self.H[sel]
            G = Hn @ np.diag(self.w) @ Hn.T
            self._cache[N] = np.diag(self.w) @ Hn.T @ np.linalg.inv(G)
        return self._cache[N]


@lru_cache(maxsize=None)
def lattice(name):
    if name == "D2Q9":
        c, w = _product_set(2)
        D = 2
    elif name == "D3Q27":
        c, w = _product_set(3)
        D = 3
    elif name == "D3Q19":
        c, w, _ = d3q19_weights()
        D = 3
    else:
        raise ValueError(f"unknown lattice {name}")
    basis = basis_indices(name)
    H = np.array([[hermite_1d(a, ci[0]) * hermite_1d(b, ci[1]) * hermite_1d(cc, ci[2])
                   for ci in c] for (a, b, cc) in basis])
    norms = (H**2) @ w
    return Lattice(name, D, c, w, CS2, basis, H, norms)


def tuple_of(k):
    """Representative index tuple (alpha_1..alpha_n) of multi-index k, e.g. (2,1,0) -> (0,0,1)."""
    return tuple(itertools.chain.from_iterable([d] * k[d] for d in range(3)))
