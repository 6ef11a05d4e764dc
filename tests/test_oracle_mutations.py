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
import test_oracle_diagnostics as TD
import test_oracle_lattice as TL
import test_oracle_lsa as TS
import test_oracle_physics as TP
from oracle import diagnostics as OD
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


def _collide_wrong_factor(lat, N, tau, f, n1=None):
    n1 = rr.f1_order(lat, N) if n1 is None else n1
    rho, u, Pi = rr.moments(lat, f)
    A = rr.offeq_second(lat, rho, u, Pi)
    f0 = rr.reconstruct(lat, N, rr.a0_coefficients(lat, N, rho, u))
    return f0 + (1.0 - tau) * rr.reconstruct(lat, n1, rr.a1_coefficients(lat, n1, A, u))  # planted: 1 - tau


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


# ---- diagnostics (Sec. 4.1 energy and enstrophy) ------------------------------

def _diag_pins():
    checks = {
        "fourier mode 3D": TD.test_vorticity_of_a_fourier_mode_3d,
        "fourier mode 2D": TD.test_vorticity_of_a_fourier_mode_2d,
        "mode enstrophy": TD.test_enstrophy_of_a_fourier_mode,
        "TGV enstrophy": lambda: TD.test_taylor_green_enstrophy_at_t0(16),
        "uniform totals": TD.test_totals_of_a_uniform_flow,
        "density wave": TD.test_totals_of_a_density_wave,
        "TGV energy": lambda: TD.test_taylor_green_energy_at_t0(8),
    }
    failed = []
    for name, fn in checks.items():
        try:
            fn()
        except (AssertionError, ValueError, IndexError):
            failed.append(name)
    return failed


def _vorticity_swapped_axis(u):
    X, Y, Z = 2, 1, 0
    if u.shape[0] == 2:
        return (OD._ddx(u[1], X) - OD._ddx(u[0], Y))[None]
    ux, uy, uz = u
    # planted: d(u_z)/dx in place of d(u_z)/dy in the x component
    return np.stack([OD._ddx(uz, X) - OD._ddx(uy, Z), OD._ddx(ux, Z) - OD._ddx(uz, X), OD._ddx(uy, X) - OD._ddx(ux, Y)])


def _vorticity_flipped_z(u):
    X, Y, Z = 2, 1, 0
    if u.shape[0] == 2:
        return (OD._ddx(u[0], Y) - OD._ddx(u[1], X))[None]  # planted: sign of w_z
    ux, uy, uz = u
    return np.stack([OD._ddx(uz, Y) - OD._ddx(uy, Z), OD._ddx(ux, Z) - OD._ddx(uz, X), OD._ddx(ux, Y) - OD._ddx(uy, X)])


def _ddx_one_sided(a, axis):
    return np.roll(a, -1, axis=axis) - a  # planted: forward difference in place of the central one


def _enstrophy_without_half(u):
    w = OD.vorticity(u)
    return float(np.mean(np.sum(w * w, axis=0)))


def _totals_without_rho_in_energy(rho, u):
    mom = [float(np.sum(rho * u[d])) for d in range(u.shape[0])]
    while len(mom) < 3:
        mom.append(0.0)
    ke = float(np.sum(0.5 * np.sum(u * u, axis=0)))  # planted: rho dropped from the energy
    return (float(np.sum(rho)), mom[0], mom[1], mom[2], ke)


def _totals_velocity_as_momentum(rho, u):
    mom = [float(np.sum(u[d])) for d in range(u.shape[0])]  # planted: sum of u, not of rho u
    while len(mom) < 3:
        mom.append(0.0)
    ke = float(np.sum(0.5 * rho * np.sum(u * u, axis=0)))
    return (float(np.sum(rho)), mom[0], mom[1], mom[2], ke)


def _ke_mean_without_half(rho, u):
    return float(np.mean(rho * np.sum(u * u, axis=0)))


DIAG_MUTATIONS = {
    "vorticity with a swapped derivative axis": ("vorticity", _vorticity_swapped_axis),
    "vorticity with the sign of w_z flipped": ("vorticity", _vorticity_flipped_z),
    "one-sided difference": ("_ddx", _ddx_one_sided),
    "enstrophy without the 1/2": ("enstrophy", _enstrophy_without_half),
    "energy without rho": ("totals", _totals_without_rho_in_energy),
    "momentum without rho": ("totals", _totals_velocity_as_momentum),
    "mean energy without the 1/2": ("kinetic_energy_mean", _ke_mean_without_half),
}


def test_unmutated_diagnostics_pass_their_pins():
    assert _diag_pins() == []


@pytest.mark.parametrize("name", list(DIAG_MUTATIONS))
def test_planted_diagnostics_mistake_is_caught(name, monkeypatch):
    attr, bad = DIAG_MUTATIONS[name]
    monkeypatch.setattr(OD, attr, bad)
    failed = _diag_pins()
    print(name, "->", failed)
    assert failed, f"no pin caught: {name}"
