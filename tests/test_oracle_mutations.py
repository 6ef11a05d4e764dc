"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case patches one plausible error into the oracle (a dropped term, a wrong
sign, a wrong index, the wrong relaxation factor, streaming the wrong way, a
transposed or non-inverted Gram matrix) and runs a quick subset of the pins;
at least one of them must fail.  The mistakes are planted in the oracle, on
the CPU, and undone after each case.
"""
import numpy as np
import pytest

import test_oracle_collision as TC
import test_oracle_lattice as TL
import test_oracle_lsa as TS
import test_oracle_physics as TP
from oracle import rr

CS2 = 1.0 / 3.0


def _quick_pins():
    """Cheap pins; returns the names of those that fail."""
    checks = {
        "appendix B 3D": lambda: TC.test_recursion_matches_appendix_b("D3Q27"),
        "appendix B 2D": lambda: TC.test_recursion_matches_appendix_b("D2Q9"),
        "pair sum": lambda: TC.test_recursion_matches_pair_sum("D3Q27"),
        "projection": lambda: TC.test_collision_projects_back_to_coefficients("D2Q9", 4),
        "fixed point": lambda: TC.test_equilibrium_is_fixed_point("D3Q27", 4),
        "uniform flow": lambda: TC.test_uniform_flow_is_fixed_point_of_full_step("D2Q9"),
        "conservation": lambda: TC.test_conservation("D2Q9", 4),
        "textbook order 2": lambda: TL.test_second_order_equilibrium_is_textbook("D2Q9"),
        "shear wave": lambda: _shear_check(),
        "advection direction": lambda: TP.test_shear_wave_is_carried_with_the_flow(),
        "LSA rest state": lambda: TS.test_rest_state_is_neutral_and_conserved_modes_have_unit_modulus(),
    }
    failed = []
    for name, fn in checks.items():
        try:
            with np.errstate(all="ignore"):
                fn()
        except (AssertionError, FloatingPointError, ValueError, IndexError, KeyError, np.linalg.LinAlgError):
            failed.append(name)
    return failed


def _shear_check():
    r = TP.shear_rate(16, 0.8, steps=200, t0=50)
    assert abs(r - 1.0) < 0.02, r


def _drop_cs2(lat, rho, u, Pi):
    A = rr._orig_offeq(lat, rho, u, Pi)
    for a in range(3):
        A[a, a] = A[a, a] + rho * CS2
    return A


def _flip_uu(lat, rho, u, Pi):
    u3 = rr._u3(u)
    A = Pi + rho * np.einsum("a...,b...->ab...", u3, u3)
    for a in range(3):
        A[a, a] = A[a, a] - rho * CS2
    return A


def _a1_drop_head(A, u3, t, memo):
    if t in memo:
        return memo[t]
    n = len(t)
    if n < 2:
        val = np.zeros_like(u3[0])
    elif n == 2:
        val = A[t[0], t[1]]
    else:
        head, last = t[:-1], t[-1]
        val = np.zeros_like(u3[0])  # planted: the a1^(n-1) u term is dropped
        for j in range(n - 1):
            term = A[head[j], last]
            for l in range(n - 1):
                if l != j:
                    term = term * u3[head[l]]
            val = val + term
    memo[t] = val
    return val


def _a1_wrong_index(A, u3, t, memo):
    if t in memo:
        return memo[t]
    n = len(t)
    if n < 2:
        val = np.zeros_like(u3[0])
    elif n == 2:
        val = A[t[0], t[1]]
    else:
        head, last = t[:-1], t[-1]
        val = _a1_wrong_index(A, u3, head, memo) * u3[last]
        for j in range(n - 1):
            term = A[head[j], head[j]]  # planted: pairs alpha_j with itself instead of alpha_n
            for l in range(n - 1):
                if l != j:
                    term = term * u3[head[l]]
            val = val + term
    memo[t] = val
    return val


def _a0_wrong_component(lat, N, rho, u):
    L = rr._lat(lat)
    u3 = rr._u3(u)
    out = []
    for r in L.kept(N):
        val = rho
        for alpha in rr.tuple_of(L.basis[r]):
            val = val * u3[(alpha + 1) % L.D]  # planted: wrong velocity component
        out.append(val)
    return np.stack(out)


def _collide_wrong_factor(lat, N, tau, f):
    rho, u, Pi = rr.moments(lat, f)
    A = rr.offeq_second(lat, rho, u, Pi)
    return rr.reconstruct(lat, N, rr.a0_coefficients(lat, N, rho, u) + (1.0 - tau) * rr.a1_coefficients(lat, N, A, u))


def _stream_backwards(lat, f):
    L = rr._lat(lat)
    out = np.empty_like(f)
    for i, (cx, cy, cz) in enumerate(L.c):
        out[i] = np.roll(f[i], shift=(-int(cz), -int(cy), -int(cx)), axis=(0, 1, 2))
    return out


def _reconstruct_without_inverse(lat, N, a):
    L = rr._lat(lat)
    sel = L.kept(N)
    Hn = L.H[sel]
    G = Hn @ np.diag(L.w) @ Hn.T
    return np.tensordot(np.diag(L.w) @ Hn.T @ G, a, axes=(1, 0))  # planted: G instead of G^-1


def _moments_diagonal_pi(lat, f):
    rho, u, Pi = rr._orig_moments(lat, f)
    for a in range(3):
        for b in range(3):
            if a != b:
                Pi[a, b] = 0.0 * Pi[a, b]  # planted: off-diagonal second moments dropped
    return rho, u, Pi


MUTATIONS = {
    "a1^(2) without the rho cs2 term": ("offeq_second", _drop_cs2),
    "a1^(2) with +rho u u": ("offeq_second", _flip_uu),
    "recursion without the a1^(n-1) u term": ("a1_tuple", _a1_drop_head),
    "recursion pairing the wrong index": ("a1_tuple", _a1_wrong_index),
    "equilibrium with the wrong velocity component": ("a0_coefficients", _a0_wrong_component),
    "collision factor 1 - tau": ("collide", _collide_wrong_factor),
    "streaming against the velocities": ("stream", _stream_backwards),
    "reconstruction with G instead of G^-1": ("reconstruct", _reconstruct_without_inverse),
    "second moment without off-diagonal terms": ("moments", _moments_diagonal_pi),
}


def test_unmutated_oracle_passes_the_quick_pins():
    assert _quick_pins() == []


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, bad = MUTATIONS[name]
    monkeypatch.setattr(rr, "_orig_offeq", rr.offeq_second, raising=False)
    monkeypatch.setattr(rr, "_orig_moments", rr.moments, raising=False)
    monkeypatch.setattr(rr, attr, bad)
    failed = _quick_pins()
    print(name, "->", failed)
    assert failed, f"no pin caught: {name}"
