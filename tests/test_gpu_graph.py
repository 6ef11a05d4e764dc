"""lb_step under HIP graph capture (torch.cuda.graph on the handle's stream).

A caller that cannot afford a launch per step captures a run of steps once and
replays it.  The step allocates nothing, synchronises nothing and records no
memset, so the capture holds only the step kernels.  The library swaps its two
state buffers at every step; a captured run of an even number of steps ends in
the buffer it started from, so the handle's own bookkeeping stays valid across
replays.  Each replay is followed by eager steps of a second handle from the
same state, a synchronisation and a bitwise comparison, three times over.
D3Q27 with FP16 or FP64 storage launches with reserved LDS (the occupancy
rule), which the capture records as well.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mlp as OM

pytestmark = pytest.mark.gpu

STEPS = 8  # even: the replayed run ends in the state buffer it started from


def _closure_weights():
    rng = np.random.default_rng(51)
    params = OM.init_params(52) + 0.02 * rng.standard_normal(OM.NPARAM).astype(np.float32)
    norm = np.concatenate([0.01 * rng.standard_normal(36), 0.02 * (1 + rng.uniform(size=36)),
                           1e-5 * rng.standard_normal(3), 1e-4 * (1 + rng.uniform(size=3))]).astype(np.float32)
    return params, norm


@pytest.mark.parametrize("case", ["d2q9-fp32", "d2q9-fp16", "d3q27-fp32", "d3q27-fp16", "d3q27-fp64", "d3q27-mom_fp32",
                                  "d2q9-closure-fp32"])
def test_graph_replays_equal_eager_steps(lbrr, gpu, case):
    torch = gpu
    lat = "D3Q27" if case.startswith("d3q27") else "D2Q9"
    storage = case.rsplit("-", 1)[1]
    shape = (20, 24, 32) if lat == "D3Q27" else (1, 72, 136)
    tau = 0.56
    rho = 1.0 + W.smooth_random(1, shape, 0.02, 61)[0]
    u = W.smooth_random(3 if lat == "D3Q27" else 2, shape, 0.05, 62)
    print(f"graph capture {case} {shape}", flush=True)
    s = torch.cuda.Stream()
    sims = []
    with torch.cuda.stream(s):
        for _ in range(2):
            sim = lbrr.Simulation(lat, shape, tau, 4, storage=storage, stream=s)
            sim.init_fields(rho, u)
            if "closure" in case:
                params, norm = _closure_weights()
                sim.set_closure(torch.from_numpy(params), torch.from_numpy(norm))
            sim.step(2)
            sims.append(sim)
    torch.cuda.synchronize()
    eager, graphed = sims
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        graphed.step(STEPS)
    torch.cuda.synchronize()
    # the capture ran nothing: both handles still hold the same state
    a, b = eager.get_populations(), graphed.get_populations()
    torch.cuda.synchronize()  # the read-outs run on the handles' stream
    assert torch.equal(a, b)
    for k in range(3):
        with torch.cuda.stream(s):
            g.replay()
            eager.step(STEPS)
        torch.cuda.synchronize()
        a, b = eager.get_populations(), graphed.get_populations()
        torch.cuda.synchronize()
        assert torch.isfinite(a).all()
        assert torch.equal(a, b), f"replay {k + 1} differs from the eager steps"
    del g
    for sim in sims:
        sim.close()
