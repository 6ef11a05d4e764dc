"""GPU parity of the resting no-slip walls (regularised Dirichlet boundary of Sec. 3.7, u_bc = 0).

Against the FP64 oracle (`oracle/walls.py`) on the same seeded inputs, with the velocity set to 0
on the wall nodes: rho, u, pi1 after several steps for every lattice and order, walls on one,
two or three axes (edges and corners included), population and moment storage, FP64 bar
1e-12 / 1e-10, FP32 1e-5 / 1e-4; FP16 population storage 2e-3 / 1e-2 (deviations with 11
significant bits, rounded at every store: measured at most 6.5e-4 on u and 3.9e-3 on pi1 after
these 16 / 6 steps); enstrophy with one-sided wall differences (FP16: 2e-4, measured 3.4e-5);
the rest state of a closed box; the channel shear mode decay rate on the GPU; argument checks.
"""
import numpy as np
import pytest

import test_gpu_parity as TP
from oracle import lattice as OL
from oracle import rr
from oracle import walls as OW

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-10), "fp32": (1e-5, 1e-4), "mom_fp64": (1e-12, 1e-10), "mom_fp32": (1e-5, 1e-4),
       "fp16": (2e-3, 1e-2)}
ENS_TOL = {"fp64": 1e-12, "mom_fp64": 1e-12, "fp32": 1e-4, "mom_fp32": 1e-4, "fp16": 2e-4}
WALLS = {2: [(True, True, False), (False, True, False), (True, False, False)],
         3: [(True, True, True), (False, True, False), (True, True, False)]}
SHAPES = {2: (1, 23, 300), 3: (7, 9, 70)}


def walled_inputs(D, shape, walls, seed):
    rho, u, pi1 = TP.smooth_inputs(D, shape, seed)
    for k, ax in ((0, 3), (1, 2), (2, 1)):
        if k < D and walls[k]:
            idx = [slice(None)] * 4
            idx[ax] = [0, shape[ax - 1] - 1]
            u[tuple(idx)] = 0.0
    return rho, u, pi1


_cache = {}


def oracle_walls(lat, N, tau, shape, walls, steps, seed):
    key = (lat, N, tau, shape, walls, steps, seed)
    if key not in _cache:
        L = OL.lattice(lat)
        rho, u, pi1 = walled_inputs(L.D, shape, walls, seed)
        f = OW.run_walls(L, N, tau, rho, u, steps, walls, rr.pi1_from_components(L, pi1))
        r, v, Pi = rr.moments(L, f)
        A = rr.pi1_components(L, rr.offeq_second(L, r, v, Pi))
        _cache[key] = (r, v, A, OW.enstrophy_walls(v, walls))
    return _cache[key]


def gpu_walls(P, lat, N, tau, shape, walls, steps, seed, storage):
    L = OL.lattice(lat)
    rho, u, pi1 = walled_inputs(L.D, shape, walls, seed)
    sim = P.Simulation(lat, shape, tau, N, storage=storage)
    sim.set_walls(*walls[: L.D])
    sim.init_fields(rho, u, pi1)
    sim.step(steps)
    r, v, p = (x.cpu().numpy() for x in sim.moments(pi1=True))
    ens = sim.enstrophy()
    sim.close()
    return r, v, p, ens


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "mom_fp64", "mom_fp32"])
@pytest.mark.parametrize("lat,N", TP.CASES)
def test_walls_parity_with_oracle(lbrr, gpu, lat, N, storage):
    L = OL.lattice(lat)
    steps = 16 if L.D == 2 else 6
    tol_ru, tol_pi = TOL[storage]
    for k, walls in enumerate(WALLS[L.D]):
        shape = SHAPES[L.D]
        print(f"walls {lat} N={N} {storage} walls={walls} shape={shape}", flush=True)
        ref = oracle_walls(lat, N, 0.63, shape, walls, steps, 40 + k)
        got = gpu_walls(lbrr, lat, N, 0.63, shape, walls, steps, 40 + k, storage)
        e = [max(TP.rel_l2(g, r), TP.rel_linf(g, r)) for g, r in zip(got[:3], ref[:3])]
        e_ens = abs(got[3] - ref[3]) / ref[3]
        print(f"  err rho {e[0]:.2e} u {e[1]:.2e} pi1 {e[2]:.2e} enstrophy {e_ens:.2e}", flush=True)
        assert e[0] <= tol_ru and e[1] <= tol_ru
        if tol_pi is not None:
            assert e[2] <= tol_pi
        assert e_ens <= ENS_TOL[storage]


@pytest.mark.parametrize("storage", ["fp64", "mom_fp64"])
@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
def test_rest_in_a_closed_box(lbrr, gpu, lat, storage):
    L = OL.lattice(lat)
    shape = (5, 6, 7) if L.D == 3 else (1, 9, 7)
    sim = lbrr.Simulation(lat, shape, 0.7, 4, storage=storage)
    sim.set_walls(True, True, L.D == 3)
    sim.init_fields(np.full(shape, 1.02), np.zeros((L.D,) + shape))
    sim.step(10)
    r, v = (x.cpu().numpy() for x in sim.moments())
    sim.close()
    assert np.abs(r - 1.02).max() <= 1e-14 and np.abs(v).max() <= 1e-15


def test_channel_mode_decay_rate_on_the_gpu(lbrr, gpu):
    """u_x = u0 sin(pi y/(ny-1)) between walls on the first and last y node decays at nu (pi/(ny-1))^2."""
    ny, nx, tau = 65, 8, 0.8
    nu = (tau - 0.5) / 3
    y = np.arange(ny)
    u = np.zeros((2, 1, ny, nx))
    u[0] = 1e-3 * np.sin(np.pi * y / (ny - 1))[None, :, None]
    sim = lbrr.Simulation("D2Q9", (1, ny, nx), tau, 4, storage="fp32")
    sim.set_walls(y=True)
    sim.init_fields(np.ones((1, ny, nx)), u)
    T = int(0.3 * (ny - 1) ** 2 / (nu * np.pi**2))
    sim.step(T // 3)
    a0 = float(sim.moments()[1][0, 0, (ny - 1) // 2, 0])
    sim.step(T - T // 3)
    a1 = float(sim.moments()[1][0, 0, (ny - 1) // 2, 0])
    sim.close()
    rate = -np.log(a1 / a0) / (T - T // 3)
    ratio = rate / (nu * (np.pi / (ny - 1)) ** 2)
    print(f"channel decay rate / theory {ratio:.6f}", flush=True)
    assert abs(ratio - 1) < 3e-4


def test_wall_arguments_are_checked(lbrr, gpu):
    sim = lbrr.Simulation("D2Q9", (1, 8, 2), 0.7, 4)
    for bad in (8, -1, 4):  # out of range, negative, z on a 2D lattice
        assert lbrr.lb_set_walls(sim.handle, bad) == lbrr.LB_ERR_INVALID_ARG
    assert lbrr.lb_set_walls(sim.handle, 1) == lbrr.LB_ERR_INVALID_ARG  # nx = 2 < 3
    assert lbrr.lb_set_walls(sim.handle, 2) == lbrr.LB_OK
    sim.close()
    sim = lbrr.Simulation("D3Q27", (4, 4, 4), 0.7, 4, storage="mom_fp32")
    assert lbrr.lb_set_walls(sim.handle, 7) == lbrr.LB_OK  # moment storage takes walls too
    sim.close()


@pytest.mark.parametrize("lz", ["1", "2", "5"])
@pytest.mark.parametrize("lat", ["D2Q9", "D3Q27"])
def test_walls_moment_storage_any_chunk_length(lbrr, gpu, monkeypatch, lat, lz):
    """Walls on every axis with FP64 moment storage at several chunk lengths (rows in 2D, z-planes
    in 3D): the wall planes and rows fall at chunk edges, inside chunks and in ragged last chunks,
    and each case matches the oracle at the FP64 bar."""
    monkeypatch.setenv("LBRR_MOM_LZ", lz)
    L = OL.lattice(lat)
    walls = (True, True, L.D == 3)
    shape = SHAPES[L.D]
    steps = 16 if L.D == 2 else 6
    ref = oracle_walls(lat, 4, 0.63, shape, walls, steps, 40)
    got = gpu_walls(lbrr, lat, 4, 0.63, shape, walls, steps, 40, "mom_fp64")
    e = [max(TP.rel_l2(g, r), TP.rel_linf(g, r)) for g, r in zip(got[:3], ref[:3])]
    print(f"walls {lat} mom_fp64 lz={lz}: err rho {e[0]:.2e} u {e[1]:.2e} pi1 {e[2]:.2e}", flush=True)
    assert e[0] <= 1e-12 and e[1] <= 1e-12 and e[2] <= 1e-10
