"""The full workloads at their full sizes and step counts, storages compared (MI355X).

* double shear layer, D2Q9 order 4, 2048^2, Re 10^4, 20000 steps: at Ma 0.2 FP32 and FP16
  population storage and FP32 moment storage against the FP64 population run; at Ma 0.5 the
  linear instability of the scheme at the local Mach numbers the flow reaches;
* random divergence-free field, D3Q19 and D3Q27 (order 4), 512^3, rms Ma 0.1, 1000 steps: FP16
  population storage and FP32 moment storage against FP32 population storage (the reference of
  this workload), throughput of each;
* 3D Taylor-Green vortex, D3Q27 order 4, 256^3, Ma 0.1 and 0.5, Re 1600, 10000 steps: FP32,
  FP16 and FP32 moment storage against the FP64 population run, pointwise before the
  transition, kinetic energy and enstrophy after it.

Bars: velocity L2 error of FP32 storages <= 1e-3 and of FP16 <= 5e-2 relative to the reference
run where the flow does not amplify perturbations; the runs must stay finite.  Throughputs and
errors are printed.
"""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def run(P, torch, lat, shape, tau, order, storage, rho, u, steps):
    sim = P.Simulation(lat, shape, tau, order, storage=storage)
    sim.init_fields(rho, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tot = np.array(sim.reduce())
    ens = sim.enstrophy()
    _, v = sim.moments()
    sim.close()
    nodes = int(np.prod(shape))
    return v, tot, ens, nodes * steps / dt / 1e9


def rel(a, b, torch):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def test_double_shear_layer_ma02_storages(lbrr, gpu):
    """Ma 0.2: every storage stays stable.  The roll-up of the shear layers amplifies any
    perturbation, so the pointwise velocity error grows with the rounding of the storage
    (FP32 and FP32 moments <= 1e-3, FP16 about 0.2 after 20000 steps); FP16's kinetic energy
    stays within 5% of the FP64 run's."""
    torch = gpu
    name = "shear_2048_ma02"
    cfg = W.WORKLOADS[name]
    n, steps = cfg["n"], cfg["steps"]
    rho, u = W.shear_layer(n, cfg["u0"], 0)
    shape = (1, n, n)
    ref = run(lbrr, torch, "D2Q9", shape, cfg["tau"], cfg["order"], "fp64", rho, u, steps)
    assert np.all(np.isfinite(ref[1]))
    assert abs(ref[1][0] - np.sum(rho)) <= 1e-10 * np.sum(rho)
    print(f"{name} fp64: {ref[3]:.1f} GLUPS, KE {ref[1][4]:.6e}, enstrophy {ref[2]:.6e}", flush=True)
    for storage in ("fp32", "mom_fp32", "fp16"):
        v, tot, ens, glups = run(lbrr, torch, "D2Q9", shape, cfg["tau"], cfg["order"], storage, rho, u, steps)
        e = rel(v, ref[0], torch)
        print(f"{name} {storage}: {glups:.1f} GLUPS, u L2 err vs fp64 {e:.2e}, KE {tot[4]:.6e}, "
              f"enstrophy {ens:.6e}", flush=True)
        assert np.all(np.isfinite(tot))
        if storage == "fp16":
            assert abs(tot[4] - ref[1][4]) <= 0.05 * ref[1][4]
        else:
            assert e <= 1e-3


_ma05 = {}


def _ma05_track(P, storage):
    """Peak |u| every 1000 steps of the Ma 0.5 shear layer, and the step of the first non-finite
    check (None if the run completes)."""
    name = "shear_2048_ma05"
    cfg = W.WORKLOADS[name]
    n, steps, every = cfg["n"], cfg["steps"], 1000
    rho, u = W.shear_layer(n, cfg["u0"], 0)
    sim = P.Simulation("D2Q9", (1, n, n), cfg["tau"], cfg["order"], storage=storage)
    sim.init_fields(rho, u)
    umax = []
    for k in range(every, steps + 1, every):
        sim.step(every)
        try:
            sim.reduce()
        except P.LBError as e:
            assert e.code == P.LB_ERR_UNSTABLE
            sim.close()
            return umax, k
        umax.append(float(sim.moments()[1].abs().max()))
    sim.close()
    return umax, None


@pytest.mark.parametrize("storage", ["fp64", "fp32", "mom_fp32", "fp16"])
def test_double_shear_layer_ma05(lbrr, gpu, storage):
    """Ma 0.5 (tau = 0.677362), 20000 steps: the rolled-up layers reach |u| ~ 0.46, where the
    order-4 D2Q9 model is linearly unstable (threshold between 0.40 and 0.45 at this tau,
    `test_oracle_lsa`).  The FP64 run must complete.  A storage whose run goes non-finite is
    reported as an expected failure (xfail) with the step and the FP64 run's peak velocity by
    then, not as a pass: the configuration is then not completed in that storage."""
    if "fp64" not in _ma05:
        _ma05["fp64"] = _ma05_track(lbrr, "fp64")
    ref, failed = _ma05["fp64"]
    print(f"shear_2048_ma05 fp64: peak |u| every 1000 steps {np.round(ref, 3).tolist()}", flush=True)
    assert failed is None
    if storage == "fp64":
        return
    umax, failed = _ma05_track(lbrr, storage)
    if failed is None:
        print(f"shear_2048_ma05 {storage}: completed 20000 steps, peak |u| {max(umax):.3f}", flush=True)
        return
    print(f"shear_2048_ma05 {storage}: non-finite by step {failed}", flush=True)
    pytest.xfail(f"{storage} goes non-finite by step {failed}, after the FP64 run's peak |u| reached "
                 f"{max(ref[: failed // 1000]):.3f} (linearly unstable above 0.40-0.45 at this tau)")


@pytest.mark.parametrize("name", ["solenoidal_512_d3q19", "solenoidal_512_d3q27"])
def test_random_field_512_storages(lbrr, gpu, name):
    torch = gpu
    cfg = W.WORKLOADS[name]
    n, steps = cfg["n"], cfg["steps"]
    rho, u = W.random_solenoidal3d(n, cfg["kmax"], cfg["urms"], 0)
    shape = (n, n, n)
    ref = run(lbrr, torch, cfg["lattice"], shape, cfg["tau"], cfg["order"], "fp32", rho, u, steps)
    print(f"{name} fp32: {ref[3]:.1f} GLUPS, KE {ref[1][4]:.6e}", flush=True)
    assert np.all(np.isfinite(ref[1]))
    for storage, bar in (("fp16", 5e-2), ("mom_fp32", 1e-3)):
        v, tot, ens, glups = run(lbrr, torch, cfg["lattice"], shape, cfg["tau"], cfg["order"], storage, rho, u, steps)
        e = rel(v, ref[0], torch)
        print(f"{name} {storage}: {glups:.1f} GLUPS, u L2 err vs fp32 {e:.2e}", flush=True)
        assert np.all(np.isfinite(tot)) and e <= bar
        del v


@pytest.mark.parametrize("name", ["tgv3d_256_ma01", "tgv3d_256_ma05"])
def test_taylor_green_256_full_run(lbrr, gpu, name):
    """10000 steps of every storage side by side with the FP64 population run (itself held to
    the oracle at 1e-12).

    * Step 2000 (t* = 2.8 at Ma 0.1, 14 at Ma 0.5): relative L2 error of u.  At Ma 0.1 the flow
      is still laminar and the errors are the rounding of each storage: FP32 and FP32 moments
      <= 1e-5, FP16 <= 1e-2.
    * Step 10000: the vortex has gone through its transition (t* = 14 at Ma 0.1, 71 at Ma 0.5),
      which amplifies any difference (at Ma 0.1 the FP32 error is 2e-7 up to step 3000 and then
      doubles about every 600 steps); the pointwise error is reported and the kinetic energy
      and enstrophy are compared: FP32 storages within 1e-5 at Ma 0.1 and 1e-3 at Ma 0.5.
      FP16 rounds every stored value to 11 significant bits at every step, a noise source at
      the grid scale that the turbulent flow keeps (measured at Ma 0.1: kinetic energy 4.5e-3,
      enstrophy 2.3e-2, a grid-scale-weighted quantity).  It is held to 1e-2 on the energy
      and 5e-2 on the enstrophy, or twice the deviation of a FP64 run whose initial velocity
      carries random relative noise of FP16's rounding size (2^-12), the spread of the flow's
      realizations, where that is larger (Ma 0.5: 5.7e-2 / 1.8e-1)."""
    torch = gpu
    cfg = W.WORKLOADS[name]
    n, steps = cfg["n"], cfg["steps"]
    rho, u = W.tgv3d(n, cfg["u0"])
    shape = (n, n, n)
    laminar = name.endswith("ma01")
    rng = np.random.default_rng(11)
    u_noisy = u * (1.0 + 2.0**-12 * rng.standard_normal(u.shape))
    runs = {}
    for st in ("fp64", "fp64_noisy", "fp32", "mom_fp32", "fp16"):
        sim = lbrr.Simulation("D3Q27", shape, cfg["tau"], cfg["order"], storage=st.split("_noisy")[0])
        sim.init_fields(rho, u_noisy if st == "fp64_noisy" else u)
        runs[st] = sim
    del u_noisy

    def u_err(st):
        _, ref = runs["fp64"].moments()
        _, v = runs[st].moments()
        e = rel(v, ref, torch)
        del v, ref
        return e

    for t in (2000, steps):
        for sim in runs.values():
            sim.step(t - sim.steps)
        errs = {st: u_err(st) for st in runs if st != "fp64"}
        print(f"{name} step {t}: u L2 err vs fp64 " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()),
              flush=True)
        if t == 2000 and laminar:
            assert errs["fp32"] <= 1e-5 and errs["mom_fp32"] <= 1e-5 and errs["fp16"] <= 1e-2
    ref_tot = np.array(runs["fp64"].reduce())
    ref_ens = runs["fp64"].enstrophy()
    dev = {}
    for st, sim in runs.items():
        tot = np.array(sim.reduce())
        assert np.all(np.isfinite(tot))
        dev[st] = (abs(tot[4] - ref_tot[4]) / ref_tot[4], abs(sim.enstrophy() - ref_ens) / ref_ens)
        print(f"{name} {st} step {steps}: KE rel diff {dev[st][0]:.2e}, enstrophy rel diff {dev[st][1]:.2e}",
              flush=True)
    for sim in runs.values():
        sim.close()
    fp32_bar = 1e-5 if laminar else 1e-3
    for st in ("fp32", "mom_fp32"):
        assert dev[st][0] <= fp32_bar and dev[st][1] <= fp32_bar
    fp16_bar = [max(floor, 2 * dev["fp64_noisy"][k]) for k, floor in ((0, 1e-2), (1, 5e-2))]
    assert dev["fp16"][0] <= fp16_bar[0] and dev["fp16"][1] <= fp16_bar[1]
