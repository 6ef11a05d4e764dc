"""Auxiliary paths of the C ABI on the GPU: checkpoint and resume, the stability
check, host-memory arguments and streams other than the default one.

* checkpoint/resume: 2n steps straight equal, bit for bit, n steps, a copy of the
  populations out of the handle (lb_get_populations), a fresh handle set from
  them (lb_set_populations) and n more steps;
* stability check (lb_set_check_interval): a NaN written into one population is
  reported by lb_step as LB_ERR_UNSTABLE at the first check after it, with the
  step counter at that check;
* host memory (on_device = 0) for lb_init_fields, lb_moments and
  lb_get/set_populations gives the same bits as device memory;
* a non-default torch stream, and a switch of stream between steps
  (lb_set_stream orders the new stream after the work on the old one), give the
  same bits as the default stream;
* poisoned destination: a step into a state buffer full of NaN writes every
  entry (plain, walled and closure steps).
"""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CASES = [("D3Q27", (6, 10, 70), 4), ("D2Q9", (1, 24, 130), 4), ("D3Q19", (5, 8, 40), 3)]


def fields(D, shape, seed):
    rho = 1.0 + W.smooth_random(1, shape, 0.02, seed)[0]
    u = W.smooth_random(D, shape, 0.06, seed + 1)
    pi1 = W.smooth_random(D * (D + 1) // 2, shape, 1e-3, seed + 2)
    return rho, u, pi1


def populations(sim):
    return sim.get_populations().cpu().numpy()


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("lat,shape,N", CASES)
def test_checkpoint_resume_is_bitwise(lbrr, gpu, lat, shape, N, storage):
    D = lbrr.DIM[lat]
    rho, u, pi1 = fields(D, shape, 11)
    n = 7
    a = lbrr.Simulation(lat, shape, 0.58, N, storage=storage)
    a.init_fields(rho, u, pi1)
    a.step(2 * n)
    straight = populations(a)
    a.close()
    b = lbrr.Simulation(lat, shape, 0.58, N, storage=storage)
    b.init_fields(rho, u, pi1)
    b.step(n)
    ckpt = b.get_populations().cpu()
    b.close()
    c = lbrr.Simulation(lat, shape, 0.58, N, storage=storage)
    c.set_populations(ckpt)
    c.step(n)
    resumed = populations(c)
    c.close()
    assert resumed.dtype == straight.dtype
    assert np.array_equal(resumed.view(np.uint8), straight.view(np.uint8))


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16"])
def test_check_interval_reports_an_injected_nan(lbrr, gpu, storage):
    torch = gpu
    lat, shape, N = "D3Q27", (4, 8, 64), 4
    rho, u, pi1 = fields(3, shape, 3)
    sim = lbrr.Simulation(lat, shape, 0.6, N, storage=storage)
    sim.init_fields(rho, u, pi1)
    sim.set_check_interval(4)
    sim.step(8)  # finite: no error
    assert sim.steps == 8
    g = sim.get_populations()
    g[13, 2, 3, 17] = float("nan")
    sim.set_populations(g)
    with pytest.raises(lbrr.LBError) as err:
        sim.step(10)
    assert err.value.code == lbrr.LB_ERR_UNSTABLE
    assert sim.steps == 12  # the first check after the NaN
    # without a check interval the step is asynchronous and does not look; lb_reduce does
    sim.set_check_interval(0)
    sim.step(3)
    with pytest.raises(lbrr.LBError) as err:
        sim.reduce()
    assert err.value.code == lbrr.LB_ERR_UNSTABLE
    sim.close()
    torch.cuda.synchronize()


def _ptr(a):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "mom_fp32"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_host_memory_arguments_match_device_memory(lbrr, gpu, storage, dtype):
    torch = gpu
    lat, shape, N = "D3Q27", (5, 9, 66), 4
    D, q = 3, 27
    np_dt = np.float64 if dtype == "f64" else np.float32
    t_dt = torch.float64 if dtype == "f64" else torch.float32
    code = lbrr.LB_F64 if dtype == "f64" else lbrr.LB_F32
    rho, u, pi1 = (np.ascontiguousarray(x.astype(np_dt)) for x in fields(D, shape, 5))

    dev = lbrr.Simulation(lat, shape, 0.61, N, storage=storage)
    dev.init_fields(torch.from_numpy(rho), torch.from_numpy(u), torch.from_numpy(pi1), dtype=t_dt)
    dev.step(5)
    r_d, u_d, p_d = dev.moments(dtype=t_dt, pi1=True)

    host = lbrr.Simulation(lat, shape, 0.61, N, storage=storage)
    lbrr.check(lbrr.lb_init_fields(host.handle, _ptr(rho), _ptr(u), _ptr(pi1), code, 0))
    host.step(5)
    r_h = np.empty(shape, np_dt)
    u_h = np.empty((D,) + shape, np_dt)
    p_h = np.empty((6,) + shape, np_dt)
    lbrr.check(lbrr.lb_moments(host.handle, _ptr(r_h), _ptr(u_h), _ptr(p_h), code, 0))
    for a, b in ((r_h, r_d), (u_h, u_d), (p_h, p_d)):
        assert np.array_equal(a, b.cpu().numpy())

    g_d = dev.get_populations().cpu().numpy()
    g_h = np.empty((q,) + shape, g_d.dtype)
    lbrr.check(lbrr.lb_get_populations(host.handle, _ptr(g_h), 0))
    assert np.array_equal(g_h.view(np.uint8), g_d.view(np.uint8))
    if not storage.startswith("mom"):
        # set from host memory, step, compare with the device handle stepped the same way
        lbrr.check(lbrr.lb_set_populations(host.handle, _ptr(g_h), 0))
        host.step(2)
        dev.step(2)
        a = np.empty_like(g_h)
        lbrr.check(lbrr.lb_get_populations(host.handle, _ptr(a), 0))
        assert np.array_equal(a.view(np.uint8), dev.get_populations().cpu().numpy().view(np.uint8))
    dev.close()
    host.close()


@pytest.mark.parametrize("storage", ["fp32", "mom_fp32"])
def test_non_default_stream_and_stream_switch(lbrr, gpu, storage):
    torch = gpu
    lat, shape, N = "D3Q27", (16, 32, 96), 4
    rho, u, pi1 = fields(3, shape, 8)
    ref = lbrr.Simulation(lat, shape, 0.57, N, storage=storage)
    ref.init_fields(rho, u, pi1)
    ref.step(40)
    want = populations(ref)
    ref.close()

    s1 = torch.cuda.Stream()
    with torch.cuda.stream(s1):
        sim = lbrr.Simulation(lat, shape, 0.57, N, storage=storage, stream=s1)
        sim.init_fields(rho, u, pi1)
        sim.step(40)
        got = populations(sim)
        sim.close()
    assert np.array_equal(got, want)

    # 20 steps on one stream, then 20 on another: the second stream must see the first 20
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s1):
        sim = lbrr.Simulation(lat, shape, 0.57, N, storage=storage, stream=s1)
        sim.init_fields(rho, u, pi1)
        sim.step(20)
    lbrr.check(lbrr.lb_set_stream(sim.handle, ctypes.c_void_p(s2.cuda_stream)))
    sim.stream = s2
    with torch.cuda.stream(s2):
        sim.step(20)
        got = populations(sim)
    sim.close()
    torch.cuda.synchronize()
    assert np.array_equal(got, want)


def _poison_cases():
    out = []
    for lat, shape, N in CASES:
        for storage in ("fp64", "fp32", "fp16"):
            for variant in ("plain", "walls") + (("closure",) if lat == "D2Q9" else ()):
                out.append(pytest.param(lat, shape, N, storage, variant, id=f"{lat}-{storage}-{variant}"))
    return out


@pytest.mark.parametrize("lat,shape,N,storage,variant", _poison_cases())
def test_every_destination_entry_is_written(lbrr, gpu, lat, shape, N, storage, variant):
    """Poisoned destination: a step into a state buffer full of NaN leaves no NaN behind.

    NaN populations and one step put NaN into both of the handle's state buffers;
    lb_set_populations then overwrites the current one with a valid state, and the
    next step writes into the poisoned one.  Every stored entry must come out finite
    and equal, bit for bit, to the same step on a fresh handle (plain step, the
    step with resting walls on every axis, and the fused closure step)."""
    torch = gpu
    from oracle import mlp as OM

    D = 2 if lat == "D2Q9" else 3
    rho, u, pi1 = fields(D, shape, 71)
    rng = np.random.default_rng(72)
    params = torch.from_numpy(OM.init_params(73) + 0.05 * rng.standard_normal(OM.NPARAM).astype(np.float32))
    norm = torch.from_numpy(np.concatenate([0.01 * rng.standard_normal(36), 0.02 * (1 + rng.uniform(size=36)),
                                            1e-5 * rng.standard_normal(3), 1e-4 * (1 + rng.uniform(size=3))])
                            .astype(np.float32))

    def configure(sim):
        if variant == "walls":
            sim.set_walls(x=True, y=True, z=D == 3)
        if variant == "closure":
            sim.set_closure(params, norm)

    ref = lbrr.Simulation(lat, shape, 0.57, N, storage=storage)
    ref.init_fields(rho, u, pi1)
    configure(ref)
    state = ref.get_populations()
    ref.step(1)
    want = populations(ref)
    sim = lbrr.Simulation(lat, shape, 0.57, N, storage=storage)
    configure(sim)
    sim.set_populations(torch.full_like(state, float("nan")))
    sim.step(1)
    assert np.isnan(populations(sim)).all()  # both buffers poisoned
    sim.set_populations(state)
    sim.step(1)
    got = populations(sim)
    assert np.isfinite(got).all()
    assert np.array_equal(got, want)
    ref.close()
    sim.close()
