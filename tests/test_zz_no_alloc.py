"""lb_reduce_static, the totals entry point that allocates nothing, against lb_reduce (GPU).

Both run the same kernels over the same partition into blocks, so the totals must be the same
bits.  Two calls in a row on different states, the second smaller, check that the static
scratch left by a call does not leak into the next; every lattice and population storage is
covered; repeated calls leave the free device memory unchanged.
"""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CASES = [("D3Q27", (40, 48, 96), 4, "fp32"), ("D2Q9", (1, 30, 70), 4, "fp64"),
         ("D3Q19", (20, 24, 50), 3, "fp16"), ("D3Q27", (9, 10, 11), 4, "fp64"),
         ("D2Q9", (1, 512, 700), 4, "fp16"), ("D3Q19", (3, 4, 5), 4, "fp32")]


def state(P, lat, shape, N, storage, seed):
    D = P.DIM[lat]
    rho = 1.0 + W.smooth_random(1, shape, 0.02, seed)[0]
    u = W.smooth_random(D, shape, 0.05, seed + 1)
    sim = P.Simulation(lat, shape, 0.6, N, storage=storage)
    sim.init_fields(rho, u)
    sim.step(3)
    return sim


def static_totals(P, torch, lat, shape, storage, pops, rho0=1.0):
    out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    nz, ny, nx = shape
    stream = torch.cuda.current_stream()
    P.check(P.lb_reduce_static(P.LATTICES[lat], P.STORAGE[storage], nx, ny, nz, rho0, ctypes.c_void_p(pops.data_ptr()),
                               ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream)))
    return tuple(out.cpu().tolist())


def test_static_totals_equal_lb_reduce_on_consecutive_calls(lbrr, gpu):
    torch = gpu
    for k, (lat, shape, N, storage) in enumerate(CASES):
        print(f"lb_reduce_static {lat} {shape} {storage}", flush=True)
        sim = state(lbrr, lat, shape, N, storage, 10 + k)
        want = sim.reduce()
        pops = sim.get_populations()
        got = static_totals(lbrr, torch, lat, shape, storage, pops)
        sim.close()
        assert got == want, (lat, shape, storage, got, want)


def test_second_smaller_call_after_a_larger_one(lbrr, gpu):
    torch = gpu
    big = state(lbrr, "D3Q27", (64, 64, 64), 4, "fp32", 3)
    small = state(lbrr, "D3Q27", (4, 5, 70), 4, "fp32", 4)
    want_big, want_small = big.reduce(), small.reduce()
    p_big, p_small = big.get_populations(), small.get_populations()
    assert static_totals(lbrr, torch, "D3Q27", (64, 64, 64), "fp32", p_big) == want_big
    assert static_totals(lbrr, torch, "D3Q27", (4, 5, 70), "fp32", p_small) == want_small
    big.close()
    small.close()


def test_repeated_calls_allocate_no_device_memory(lbrr, gpu):
    torch = gpu
    sim = state(lbrr, "D3Q27", (16, 16, 64), 4, "fp32", 8)
    pops = sim.get_populations()
    out = torch.empty(5, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    args = (lbrr.LATTICES["D3Q27"], lbrr.STORAGE["fp32"], 64, 16, 16, 1.0, ctypes.c_void_p(pops.data_ptr()),
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    lbrr.check(lbrr.lb_reduce_static(*args))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(200):
        lbrr.check(lbrr.lb_reduce_static(*args))
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert tuple(out.cpu().tolist()) == sim.reduce()
    sim.close()


def test_moment_storage_is_rejected(lbrr, gpu):
    torch = gpu
    pops = torch.zeros((27, 2, 2, 2), dtype=torch.float32, device="cuda")
    out = torch.empty(5, dtype=torch.float64, device="cuda")
    code = lbrr.lb_reduce_static(lbrr.LATTICES["D3Q27"], lbrr.STORAGE["mom_fp32"], 2, 2, 2, 1.0,
                                 ctypes.c_void_p(pops.data_ptr()), ctypes.c_void_p(out.data_ptr()), None)
    assert code == lbrr.LB_ERR_UNSUPPORTED
    assert np.isfinite(0.0)
