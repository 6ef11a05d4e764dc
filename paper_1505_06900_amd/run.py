"""Run one of the named workloads on the GPU and print a JSON record per report.

    python -m paper_1505_06900_amd.run NAME [--storage fp32|fp16|fp64|mom_fp32|mom_fp64]
                                            [--steps N] [--report-every K] [--seed S]

NAME is a key of workloads.WORKLOADS with an initial-field recipe (the Taylor-Green
vortices, the double shear layers, the random fields, the fine decaying-turbulence
run).  Every K steps (and at the end) one JSON line: the step count, the GLUPS of
the steps since the previous line (HIP events on the handle's stream), the FP64
totals (mass, momentum, kinetic energy) and the enstrophy.  --steps defaults to
the workload's own step count.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("name")
    ap.add_argument("--storage", default="fp32", choices=["fp64", "fp32", "fp16", "mom_fp64", "mom_fp32"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--report-every", type=int, default=None)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch

    import workloads as W

    from . import Simulation

    if a.name not in W.WORKLOADS:
        ap.error(f"unknown workload {a.name}; known: {', '.join(sorted(W.WORKLOADS))}")
    cfg = W.WORKLOADS[a.name]
    rho, u, shape = W.initial_fields(a.name, a.seed)
    steps = a.steps if a.steps is not None else cfg.get("steps", 1000)
    every = a.report_every if a.report_every is not None else max(steps, 1)
    if steps < 0 or every < 1:
        ap.error("--steps must be >= 0 and --report-every >= 1")
    sim = Simulation(cfg["lattice"], shape, cfg["tau"], cfg["order"], storage=a.storage)
    sim.init_fields(rho, u)
    nodes = shape[0] * shape[1] * shape[2]
    done = 0

    def record(glups):
        mass, px, py, pz, ke = (float(v) for v in sim.reduce())
        return {"workload": a.name, "lattice": cfg["lattice"], "order": cfg["order"], "storage": a.storage,
                "shape": list(shape), "tau": cfg["tau"], "step": done, "glups": glups, "mass": mass,
                "momentum": [px, py, pz], "kinetic_energy": ke, "enstrophy": float(sim.enstrophy())}

    print(json.dumps(record(None)), flush=True)
    while done < steps:
        k = min(every, steps - done)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step(k)
        e1.record(sim.stream)
        e1.synchronize()
        done += k
        print(json.dumps(record(nodes * k / (e0.elapsed_time(e1) * 1e-3) / 1e9)), flush=True)
    sim.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
