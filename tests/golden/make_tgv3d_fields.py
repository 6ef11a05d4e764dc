"""Write the FP64 oracle's rho and u of the 3D Taylor-Green vortex at sampled nodes.

D3Q27 order 4, 64^3, Re 1600 on L = N/(2 pi), Ma 0.1 (relaxation time of
workloads.WORKLOADS "tgv3d_64_ma01"), after 100 and 500 steps.  The nodes are
the eight corners of the box and 504 nodes drawn with numpy's default_rng(2024).
Calls only the oracle and the input generators; the output file
tests/golden/tgv3d_64_ma01_fields.txt holds one line per (step, node):
step, z, y, x, rho, u_x, u_y, u_z, as written by this script.

usage: python tests/golden/make_tgv3d_fields.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import lattice as OL  # noqa: E402
from oracle import rr  # noqa: E402

STEPS = (100, 500)
NRANDOM = 504


def sample_nodes(n):
    rng = np.random.default_rng(2024)
    pts = rng.integers(0, n, size=(NRANDOM, 3))
    corners = np.array([[z, y, x] for z in (0, n - 1) for y in (0, n - 1) for x in (0, n - 1)])
    return np.concatenate([corners, pts])


def main():
    cfg = W.WORKLOADS["tgv3d_64_ma01"]
    n, tau, order = cfg["n"], cfg["tau"], cfg["order"]
    L = OL.lattice(cfg["lattice"])
    rho, u = W.tgv3d(n, cfg["u0"])
    f = rr.init_populations(L, order, rho, u)
    pts = sample_nodes(n)
    idx = tuple(pts.T)
    out = os.path.join(HERE, "tgv3d_64_ma01_fields.txt")
    with open(out, "w") as fh:
        fh.write(f"# FP64 oracle, D3Q27 order {order}, {n}^3 TGV, u0 {cfg['u0']:.8f}, tau {tau}, Re 1600\n")
        fh.write("# written by tests/golden/make_tgv3d_fields.py; columns: step, z, y, x, rho, u_x, u_y, u_z\n")
        t = 0
        for target in STEPS:
            while t < target:
                f = rr.step(L, order, tau, f)
                t += 1
                if t % 50 == 0:
                    print("step", t, flush=True)
            r, v, _ = rr.moments(L, f)
            for k, (z, y, x) in enumerate(pts):
                vals = (r[idx][k], v[0][idx][k], v[1][idx][k], v[2][idx][k])
                fh.write(f"{t} {z} {y} {x} " + " ".join(f"{a:.17e}" for a in vals) + "\n")
            fh.flush()
    assert np.isfinite(f).all()


if __name__ == "__main__":
    main()
