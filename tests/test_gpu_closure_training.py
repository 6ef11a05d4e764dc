"""The trained closure against the method without it (decaying 2D turbulence, D2Q9).

Fine 1024^2 (tau_f 0.535472) and coarse 256^2 (tau_c 0.508868) runs of random
vorticity with 4 <= |k| <= 12, rms Ma 0.1, Re 5000; training seeds 0-3
(40 snapshots each, every 200 fine steps), held-out seed 4.  The network is
trained on the GPU by the library's own forward/backward/Adam kernels
(3000 steps, batch 4096).  Asserted: held-out a-priori skill, a stable
closure run, and a lower velocity error than the plain coarse run against
the coarse-grained fine run at every checkpoint after the first, over 2000
coarse steps.  Printed: the error curves and the step-cost ratio.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_trained_closure_beats_plain_coarse_run(lbrr, gpu):
    torch = gpu
    from paper_1505_06900_amd import closure as C

    cf, cc = dict(W.WORKLOADS["turb2d_fine_1024"]), dict(W.WORKLOADS["turb2d_coarse_256"])
    xs, ys = [], []
    for seed in range(4):
        x, y = C.generate(seed, cf, cc, snapshots=40, interval=200)
        xs.append(x)
        ys.append(y)
    x, y = torch.cat(xs), torch.cat(ys)
    del xs, ys
    xt, yt = C.generate(4, cf, cc, snapshots=20, interval=200)
    norm = C.norm_stats(x, y)
    params, losses = C.train(x, y, norm, steps=3000, batch=4096, lr=1e-3, seed=0)
    print("losses", losses, flush=True)
    assert losses[-1][1] < 0.02  # normalised mean squared error (1 = predicting the mean)
    r2 = C.r2_score(C.predict(params, norm, xt), yt)
    print("held-out R2", r2, flush=True)
    assert np.all(r2 > 0.9)
    res = C.a_posteriori(params, norm, 4, cf, cc, coarse_steps=2000, every=200)
    ep, ec = np.array(res["err_u"]["plain"]), np.array(res["err_u"]["closure"])
    print("err plain  ", np.round(ep, 5).tolist(), flush=True)
    print("err closure", np.round(ec, 5).tolist(), flush=True)
    print("KE fine/plain/closure", [np.round(res["ke"][k][-1], 8) for k in ("fine", "plain", "closure")])
    print("enstrophy fine/plain/closure", [np.round(res["enstrophy"][k][-1], 10) for k in ("fine", "plain", "closure")])
    print("step ms", res["step_ms"], "cost ratio", res.get("cost_ratio"), flush=True)
    assert res["stable"]["closure"] and res["stable"]["plain"]
    assert np.all(ec[1:] < ep[1:])
    assert ec[-1] < 0.9 * ep[-1]
