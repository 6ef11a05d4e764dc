"""GPU parity of the learned-closure kernels against the FP64 closure oracle.

Bars: coarse-graining 1e-12 (FP64 in, FP64 out); features 1e-6 relative to
their scale (FP32 outputs of an FP64 state); MLP outputs within 2e-3 of the
oracle at the worst sample and 1e-5 at the median (same BF16 rounding points,
FP32 vs FP64 accumulation: a rare one-ulp BF16 flip of an activation moves an
output by about 2^-8 of its size); the batch gradient within 1e-3 relative
(measured 1.3e-4) and each layer's block within 2e-3; Adam 1e-6; the fused
closure step with a zero network equals the plain step, and with a random
network matches the oracle collision with the predicted correction added to
a1^(2).
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import closure as OC
from oracle import lattice as OL
from oracle import mlp as OM
from oracle import rr

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _s(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def rand_norm(rng, scale_y=1e-4):
    xm = 0.01 * rng.standard_normal(36)
    xs = 0.02 * (1 + rng.uniform(size=36))
    ym = scale_y * 0.1 * rng.standard_normal(3)
    ys = scale_y * (1 + rng.uniform(size=3))
    return np.concatenate([xm, xs, ym, ys]).astype(np.float32)


def oracle_forward(params, norm, x):
    n = norm.astype(np.float64)
    xn = (x.astype(np.float64) - n[:36]) / n[36:72]
    y, _ = OM.forward(params.astype(np.float64), xn, rounding=True)
    return y * n[75:78] + n[72:75]


def test_coarsen_matches_oracle(lbrr, gpu):
    torch = gpu
    from paper_1505_06900_amd import closure as C

    ny, nx, F = 48, 64, 4
    rho = 1.0 + W.smooth_random(1, (1, ny, nx), 0.02, 1)[0]  # (1, ny, nx)
    u = W.smooth_random(2, (1, ny, nx), 0.05, 2)  # (2, 1, ny, nx)
    pi1 = W.smooth_random(3, (1, ny, nx), 1e-3, 3)  # (3, 1, ny, nx)
    for alpha, beta in [C.state_factors(0.6, 0.52, "onestep"), C.state_factors(0.6, 0.52, "flux"),
                        (0.0, C.flux_label_factor(0.52))]:
        rc, uc, pc = C.coarsen(*(torch.from_numpy(a).cuda() for a in (rho, u, pi1)), F, alpha, beta)
        r_ref, u_ref, p_ref = OC.coarse_grain(rho[0], u[:, 0], pi1[:, 0], F, alpha, beta)
        np.testing.assert_allclose(rc.cpu().numpy()[0], r_ref, rtol=1e-13)
        np.testing.assert_allclose(uc.cpu().numpy()[:, 0], u_ref, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(pc.cpu().numpy()[:, 0], p_ref, rtol=1e-10, atol=1e-16)
    # the one-step target is the oracle's coarse_target
    _, _, pc = C.coarsen(*(torch.from_numpy(a).cuda() for a in (rho, u, pi1)), F, *C.state_factors(0.6, 0.52, "onestep"))
    np.testing.assert_allclose(pc.cpu().numpy()[:, 0], OC.coarse_target(rho[0], u[:, 0], pi1[:, 0], 0.6, 0.52, F)[2],
                               rtol=1e-10, atol=1e-15)


def test_features_match_oracle(lbrr, gpu):
    torch = gpu
    L = OL.lattice("D2Q9")
    ny, nx = 20, 70
    rho, u, pi1 = (1.0 + W.smooth_random(1, (1, ny, nx), 0.02, 4)[0], W.smooth_random(2, (1, ny, nx), 0.06, 5),
                   W.smooth_random(3, (1, ny, nx), 1e-3, 6))
    g = rr.collide(L, 4, 0.7, rr.init_populations(L, 4, rho, u, rr.pi1_from_components(L, pi1)))
    g = g + W.noise(g.shape, 1e-4, 7) * L.w[:, None, None, None]
    sim = lbrr.Simulation("D2Q9", (1, ny, nx), 0.7, 4, storage="fp64")
    sim.set_populations(torch.from_numpy(g - L.w[:, None, None, None]))
    target = W.smooth_random(3, (1, ny, nx), 1e-3, 8)
    feat, lab = sim.closure_features(a_target=torch.from_numpy(target).cuda())
    X, Ap = OC.features(g)
    scale = np.abs(X).max(axis=0)
    np.testing.assert_allclose(feat.cpu().numpy(), X, atol=1e-6 * scale.max())
    lab_ref = target.reshape(3, -1).T - Ap
    np.testing.assert_allclose(lab.cpu().numpy(), lab_ref, atol=1e-7 * np.abs(lab_ref).max() + 1e-12)
    sim.close()


def test_mlp_forward_matches_oracle(lbrr, gpu):
    torch = gpu
    rng = np.random.default_rng(11)
    params = OM.init_params(12) + 0.02 * rng.standard_normal(OM.NPARAM).astype(np.float32)
    norm = rand_norm(rng)
    n = 1000  # not a multiple of the 128-sample block: ragged tail
    x = (norm[:36] + norm[36:72] * rng.standard_normal((n, 36))).astype(np.float32)
    y = torch.empty((n, 3), device="cuda", dtype=torch.float32)
    pt, nt, xt = (torch.from_numpy(a).cuda() for a in (params, norm, x))
    lbrr.check(lbrr.lb_mlp_forward(_p(pt), _p(nt), _p(xt), n, _p(y), _s(torch)))
    ref = oracle_forward(params, norm, x)
    got = y.cpu().numpy()
    err = np.abs(got - ref)
    scale = np.abs(ref - norm[72:75]).max()
    print(f"forward max err {err.max() / scale:.2e}, median {np.median(err) / scale:.2e}")
    assert err.max() <= 2e-3 * scale
    assert np.median(err) <= 1e-5 * scale


def test_mlp_gradient_and_adam_match_oracle(lbrr, gpu):
    torch = gpu
    rng = np.random.default_rng(21)
    params = OM.init_params(22) + 0.02 * rng.standard_normal(OM.NPARAM).astype(np.float32)
    norm = rand_norm(rng)
    N, B = 3000, 200  # batch not a multiple of the 32-sample block
    x = (norm[:36] + norm[36:72] * rng.standard_normal((N, 36))).astype(np.float32)
    t = (norm[72:75] + norm[75:78] * rng.standard_normal((N, 3))).astype(np.float32)
    idx = rng.integers(0, N, size=B).astype(np.int32)
    pt, nt, xt, tt, it = (torch.from_numpy(a).cuda() for a in (params, norm, x, t, idx))
    g = torch.empty(OM.NPARAM, device="cuda", dtype=torch.float32)
    loss = torch.empty(1, device="cuda", dtype=torch.float32)
    lbrr.check(lbrr.lb_mlp_gradient(_p(pt), _p(nt), _p(xt), _p(tt), N, _p(it), B, _p(g), _p(loss), _s(torch)))
    g1 = g.cpu().numpy().copy()
    lbrr.check(lbrr.lb_mlp_gradient(_p(pt), _p(nt), _p(xt), _p(tt), N, _p(it), B, _p(g), _p(loss), _s(torch)))
    assert np.array_equal(g1, g.cpu().numpy())  # fixed-order reduction: bitwise reproducible
    n64 = norm.astype(np.float64)
    xn = (x[idx].astype(np.float64) - n64[:36]) / n64[36:72]
    tn = (t[idx].astype(np.float64) - n64[72:75]) / n64[75:78]
    l_ref, g_ref = OM.backward(params.astype(np.float64), xn, tn, rounding=True)
    rel = np.linalg.norm(g1 - g_ref) / np.linalg.norm(g_ref)
    print(f"loss gpu {loss.item():.6f} oracle {l_ref:.6f}; gradient rel err {rel:.2e}")
    assert loss.item() == pytest.approx(l_ref, rel=1e-3)
    assert rel <= 1e-3
    for name, (o, n) in {"W1": (0, 2304), "b1": (2304, 2368), "W2": (2368, 6464), "b2": (6464, 6528),
                         "W3": (6528, 6720), "b3": (6720, 6723)}.items():
        r = np.linalg.norm(g1[o:n] - g_ref[o:n]) / np.linalg.norm(g_ref[o:n])
        print(f"  {name} rel err {r:.2e}")
        assert r <= 2e-3, (name, r)
    # Adam, two steps
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    pm, mm, vm = params.astype(np.float64), np.zeros(OM.NPARAM), np.zeros(OM.NPARAM)
    for step in (1, 2):
        lbrr.check(lbrr.lb_mlp_adam(_p(pt), _p(m), _p(v), _p(g), step, 1e-3, 0.9, 0.999, 1e-8, _s(torch)))
        pm, mm, vm = OM.adam(pm, mm, vm, g1.astype(np.float64), step)
    np.testing.assert_allclose(pt.cpu().numpy(), pm, rtol=1e-5, atol=1e-7)


def _oracle_closure_step(g, params, norm, tau):
    L = OL.lattice("D2Q9")
    X, _ = OC.features(g)
    d = oracle_forward(params, norm, X)  # (nodes, 3)
    f = rr.stream(L, g)
    rho, u, Pi = rr.moments(L, f)
    A = rr.offeq_second(L, rho, u, Pi)
    ny, nx = g.shape[-2:]
    A[0, 0] += d[:, 0].reshape(1, ny, nx)
    A[0, 1] += d[:, 1].reshape(1, ny, nx)
    A[1, 0] += d[:, 1].reshape(1, ny, nx)
    A[1, 1] += d[:, 2].reshape(1, ny, nx)
    a0 = rr.a0_coefficients(L, 4, rho, u)
    a1 = rr.a1_coefficients(L, 4, A, u)
    return rr.reconstruct(L, 4, a0 + (1 - 1 / tau) * a1), d


@pytest.mark.parametrize("wpr", ["1", "2"])
@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("ny,nx", [(24, 200), (25, 130), (3, 10), (1, 70)])
def test_fused_closure_step(lbrr, gpu, storage, ny, nx, wpr, monkeypatch):
    """Rows of 4 and 3 tiles of 64 columns with ragged ends; the fused step's blocks cover 4 rows,
    so at ny = 25 the last block row holds one row of the grid and three past it.  The tiny
    periodic boxes (3 x 10, 1 x 70) wrap the neighbour halo several times over.  Three more
    steps check the state carried from one closure step to the next.  Both launch forms of the
    fused step: one wave per row and two (the form the library takes on grids of at most one
    block per compute unit; FP64 storage always takes one).

    FP16 storage: the oracle starts from the FP16-rounded deviations the library stores, and the
    bar adds one FP16 rounding of the stored outputs (2^-11 of the largest deviation)."""
    torch = gpu
    monkeypatch.setenv("LBRR_CLOSURE_WPR", wpr)
    L = OL.lattice("D2Q9")
    tau = 0.58
    rho, u, pi1 = (1.0 + W.smooth_random(1, (1, ny, nx), 0.02, 31)[0], W.smooth_random(2, (1, ny, nx), 0.06, 32),
                   W.smooth_random(3, (1, ny, nx), 1e-3, 33))
    wr = L.w[:, None, None, None]
    g = rr.collide(L, 4, tau, rr.init_populations(L, 4, rho, u, rr.pi1_from_components(L, pi1)))
    if storage == "fp16":
        g = wr + (g - wr).astype(np.float16).astype(np.float64)
    rng = np.random.default_rng(34)
    norm = rand_norm(rng, scale_y=2e-4)
    # (a) zero output layer and zero output mean: the plain step exactly
    zero = OM.init_params(35)
    zero[6528:] = 0.0
    nz_ = norm.copy()
    nz_[72:75] = 0.0
    plain = lbrr.Simulation("D2Q9", (1, ny, nx), tau, 4, storage=storage)
    plain.set_populations(torch.from_numpy(g - wr))
    plain.step(1)
    clos = lbrr.Simulation("D2Q9", (1, ny, nx), tau, 4, storage=storage)
    clos.set_populations(torch.from_numpy(g - wr))
    clos.set_closure(torch.from_numpy(zero), torch.from_numpy(nz_))
    clos.step(1)
    a, b = (x.cpu().numpy().astype(np.float64) for x in (plain.get_populations(), clos.get_populations()))
    tol = 1e-15 if storage == "fp64" else 1e-7
    assert np.abs(a - b).max() <= tol * np.abs(a).max()
    # (b) random network vs the oracle
    params = OM.init_params(36) + 0.05 * rng.standard_normal(OM.NPARAM).astype(np.float32)
    clos.set_populations(torch.from_numpy(g - wr))
    clos.set_closure(torch.from_numpy(params), torch.from_numpy(norm))
    clos.step(1)
    got = clos.get_populations().cpu().numpy().astype(np.float64)
    ref, _ = _oracle_closure_step(g, params, norm, tau)
    effect = np.abs(ref - rr.step_post(L, 4, tau, g)).max()  # the correction must matter
    err = np.abs(got - (ref - wr)).max()
    store = {"fp64": 1e-14, "fp32": 1e-7, "fp16": 2.0**-11 * np.abs(ref - wr).max()}[storage]
    print(f"closure effect {effect:.3e}, gpu-oracle {err:.3e}, storage rounding allowance {store:.1e}")
    assert effect > 1e-6
    assert err <= 2e-3 * effect + store
    # three more closure steps from the state reached (the oracle from its own state)
    for _ in range(3):
        clos.step(1)
        ref, _ = _oracle_closure_step(ref, params, norm, tau)
    got = clos.get_populations().cpu().numpy().astype(np.float64)
    err4 = np.abs(got - (ref - wr)).max()
    print(f"  after 4 closure steps: gpu-oracle {err4:.3e}")
    assert err4 <= 4 * (2e-3 * effect + store)
    plain.close()
    clos.close()


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
@pytest.mark.parametrize("ny,nx", [(25, 130), (64, 64)])
def test_fused_closure_launch_forms_agree_bitwise(lbrr, gpu, storage, ny, nx, monkeypatch):
    """The two launch forms of the fused step (one and two waves per row) compute every
    sample's features, products and activations in the same order, so five steps from the
    same state give the same bits; an out-of-range LBRR_CLOSURE_WPR is ignored (the
    library's own choice, also the same bits)."""
    torch = gpu
    L = OL.lattice("D2Q9")
    tau = 0.55
    rho, u = 1.0 + W.smooth_random(1, (1, ny, nx), 0.02, 41)[0], W.smooth_random(2, (1, ny, nx), 0.06, 42)
    g = rr.init_populations(L, 4, rho, u)
    wr = L.w[:, None, None, None]
    rng = np.random.default_rng(43)
    params = OM.init_params(44) + 0.05 * rng.standard_normal(OM.NPARAM).astype(np.float32)
    norm = rand_norm(rng, scale_y=2e-4)
    out = {}
    for wpr in ("1", "2", "7"):
        monkeypatch.setenv("LBRR_CLOSURE_WPR", wpr)
        sim = lbrr.Simulation("D2Q9", (1, ny, nx), tau, 4, storage=storage)
        sim.set_populations(torch.from_numpy(g - wr))
        sim.set_closure(torch.from_numpy(params), torch.from_numpy(norm))
        sim.step(5)
        out[wpr] = sim.get_populations().cpu().numpy()
        sim.close()
    assert np.isfinite(out["1"]).all()
    assert np.array_equal(out["1"], out["2"])
    assert np.array_equal(out["1"], out["7"])
