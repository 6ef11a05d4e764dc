"""Write the FP64 oracle's kinetic-energy and enstrophy curves of the 3D Taylor-Green vortex.

D3Q27 order 4, 64^3, Re 1600 on L = N/(2 pi), Ma 0.1 and 0.5 (relaxation times of
workloads.WORKLOADS "tgv3d_64_ma01" / "tgv3d_64_ma05"), 2500 steps, values every
50 steps.  Calls only the oracle and the input generators; the output files
tests/golden/tgv3d_64_<case>_curves.txt hold: step, mean kinetic energy,
mean enstrophy (volume means), as written by this script.

usage: python tests/golden/make_tgv3d_curves.py ma01|ma05
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import diagnostics as OD  # noqa: E402
from oracle import lattice as OL  # noqa: E402
from oracle import rr  # noqa: E402


def main(case):
    cfg = W.WORKLOADS[f"tgv3d_64_{case}"]
    n, tau, order, steps = cfg["n"], cfg["tau"], cfg["order"], cfg["steps"]
    L = OL.lattice(cfg["lattice"])
    rho, u = W.tgv3d(n, cfg["u0"])
    f = rr.init_populations(L, order, rho, u)
    out = os.path.join(HERE, f"tgv3d_64_{case}_curves.txt")
    with open(out, "w") as fh:
        fh.write(f"# FP64 oracle, D3Q27 order {order}, {n}^3 TGV, u0 {cfg['u0']:.8f}, tau {tau}, Re 1600\n")
        fh.write("# written by tests/golden/make_tgv3d_curves.py; columns: step, mean KE, mean enstrophy\n")
        for t in range(steps + 1):
            if t % 50 == 0:
                r, v, _ = rr.moments(L, f)
                fh.write(f"{t} {OD.kinetic_energy_mean(r, v):.17e} {OD.enstrophy(v):.17e}\n")
                fh.flush()
                print(case, t, flush=True)
            if t < steps:
                f = rr.step(L, order, tau, f)
    assert np.isfinite(f).all()


if __name__ == "__main__":
    main(sys.argv[1])
