"""3D Taylor-Green vortex (D3Q27 order 4, 64^3, Re 1600, Ma 0.1 and 0.5): kinetic-energy and
enstrophy curves of the GPU runs against the FP64 oracle's curves over 2500 steps.

The oracle curves are stored in tests/golden/tgv3d_64_<case>_curves.txt, written by
tests/golden/make_tgv3d_curves.py (oracle only).  Bars (largest relative deviation
over the curve): FP64 storage 1e-9; FP32 5e-4, from the rounding drift of the
stored FP32 state (velocity error growing by about 6e-8 per step, so about
1.5e-4 after 2500 steps and twice that in the quadratic kinetic energy);
FP16 2e-2; the enstrophy, a derivative quantity, gets 5 times the bar.
"""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = {"fp64": 1e-9, "fp32": 5e-4, "fp16": 2e-2, "mom_fp64": 1e-9, "mom_fp32": 5e-4}


def load(case):
    d = np.loadtxt(os.path.join(GOLDEN, f"tgv3d_64_{case}_curves.txt"))
    return d[:, 0].astype(int), d[:, 1], d[:, 2]


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "mom_fp64", "mom_fp32"])
@pytest.mark.parametrize("case", ["ma01", "ma05"])
def test_tgv3d_curves_match_oracle(lbrr, gpu, case, storage):
    cfg = W.WORKLOADS[f"tgv3d_64_{case}"]
    n = cfg["n"]
    steps, ke_ref, ens_ref = load(case)
    rho, u = W.tgv3d(n, cfg["u0"])
    sim = lbrr.Simulation("D3Q27", (n, n, n), cfg["tau"], cfg["order"], storage=storage)
    sim.init_fields(rho, u)
    ke, ens = [], []
    for t in steps:
        sim.step(int(t) - sim.steps)
        ke.append(sim.reduce()[4] / n**3)
        ens.append(sim.enstrophy())
    sim.close()
    e_ke = np.max(np.abs(np.array(ke) - ke_ref) / ke_ref)
    e_en = np.max(np.abs(np.array(ens) - ens_ref) / ens_ref)
    print(f"TGV3D {case} {storage}: max rel dev KE {e_ke:.2e} enstrophy {e_en:.2e}; "
          f"KE(end)/KE(0) {ke[-1] / ke[0]:.5f}, enstrophy peak at step {steps[int(np.argmax(ens))]}", flush=True)
    assert e_ke <= TOL[storage]
    assert e_en <= 5 * TOL[storage]
