"""GPU parity of the moment-state storage (rho - rho0, rho u, a1^(2) per node).

The collision of Sec. 3.5 leaves every population a function of its node's
rho, u and a1^(2), so storing those moments and rebuilding the populations at
the source node before streaming is the same update.  Checked against the FP64
oracle (which stores populations) on the same seeded inputs:

  rho, u, pi1   same bars as the population storage (FP64 1e-12 / 1e-10,
                FP32 1e-5 / 1e-4), every lattice and order, shapes that span
                several blocks (62 x 6 target nodes per FP32 block, 30 x 6
                FP64) with ragged tails and several z-chunks with a ragged
                last chunk;
  populations   the post-collision deviations rebuilt by lb_get_populations
                equal the oracle's collide(f) - w rho0 (FP64: 1e-13 at t = 0,
                the FP64 bar 1e-12 after three steps);
  cross-check   FP64 moment and population storage on the GPU agree on rho, u,
                totals and enstrophy of a 3D Taylor-Green run;
  chunking      the z-chunk length does not change a single bit;
  edges         boxes of 1 to 3 nodes along an axis (periodic images of one
                node fill a block), block-boundary widths of the FP64 and
                FP32 tiles.
"""
import numpy as np
import pytest

import test_gpu_parity as TP
import workloads as W
from oracle import lattice as OL
from oracle import rr

pytestmark = pytest.mark.gpu

TOL = {"mom_fp64": (1e-12, 1e-10), "mom_fp32": (1e-5, 1e-4)}
SHAPES = {2: [(1, 37, 70), (1, 9, 300)], 3: [(13, 10, 70), (12, 14, 20)]}


def errs(got, ref):
    return [max(TP.rel_l2(g, r), TP.rel_linf(g, r)) for g, r in zip(got, ref)]


@pytest.mark.parametrize("storage", ["mom_fp64", "mom_fp32"])
@pytest.mark.parametrize("lat,N", TP.CASES)
def test_moment_storage_parity_with_oracle(lbrr, gpu, monkeypatch, lat, N, storage):
    D = lbrr.DIM[lat]
    steps = 24 if D == 2 else 8
    tau = 0.62
    tol_ru, tol_pi = TOL[storage]
    monkeypatch.setenv("LBRR_MOM_LZ", "4")  # 13 planes -> chunks of 4, 4, 4, 1
    for k, shape in enumerate(SHAPES[D]):
        print(f"case {lat} N={N} {storage} shape={shape} steps={steps}", flush=True)
        ref = TP.oracle_run(lat, N, tau, shape, steps, 100 + k)
        got = TP.gpu_run(lbrr, lat, N, tau, shape, steps, 100 + k, storage)
        e_rho, e_u, e_pi = errs(got, ref)
        print(f"  err rho {e_rho:.2e} u {e_u:.2e} pi1 {e_pi:.2e}", flush=True)
        assert e_rho <= tol_ru and e_u <= tol_ru and e_pi <= tol_pi


@pytest.mark.parametrize("lat,N", TP.CASES)
def test_rebuilt_populations_match_oracle(lbrr, gpu, lat, N):
    """lb_get_populations of the moment state = the oracle's post-collision deviations, at t = 0
    and after three steps."""
    L = OL.lattice(lat)
    shape = (1, 11, 67) if L.D == 2 else (5, 7, 66)
    rho, u, pi1 = TP.smooth_inputs(L.D, shape, 7)
    tau = 0.7
    wr = L.w.reshape((-1, 1, 1, 1))
    f = rr.init_populations(L, N, rho, u, rr.pi1_from_components(L, pi1))
    sim = lbrr.Simulation(lat, shape, tau, N, storage="mom_fp64")
    sim.init_fields(rho, u, pi1)
    for steps in (0, 3):
        for _ in range(steps):
            f = rr.step(L, N, tau, f)
        sim.step(steps)
        ref = rr.collide(L, N, tau, f) - wr
        got = sim.get_populations().cpu().numpy()
        e = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"{lat} N={N} t={sim.steps}: populations rel err {e:.2e}", flush=True)
        assert e <= (1e-13 if steps == 0 else 1e-12)  # rounding of two FP64 formulations accumulates
    sim.close()


def test_moment_and_population_storage_agree(lbrr, gpu):
    """FP64 population and moment storage on the GPU: a 3D Taylor-Green run, D3Q27 order 4."""
    n, u0, tau = 32, 0.05, 0.52
    rho, u = W.tgv3d(n, u0)
    out = {}
    for storage in ("fp64", "mom_fp64"):
        sim = lbrr.Simulation("D3Q27", (n, n, n), tau, 4, storage=storage)
        sim.init_fields(rho, u)
        sim.step(60)
        r, v, p = (x.cpu().numpy() for x in sim.moments(pi1=True))
        out[storage] = (r, v, p, np.array(sim.reduce()), sim.enstrophy())
        sim.close()
    a, b = out["fp64"], out["mom_fp64"]
    e = errs(b[:3], a[:3])
    print(f"moment vs population FP64: rho {e[0]:.2e} u {e[1]:.2e} pi1 {e[2]:.2e}", flush=True)
    assert e[0] <= 1e-12 and e[1] <= 1e-12 and e[2] <= 1e-10
    tot_a, tot_b = a[3], b[3]
    assert abs(tot_b[0] - tot_a[0]) <= 1e-12 * abs(tot_a[0])
    assert np.abs(tot_b[1:4] - tot_a[1:4]).max() <= 1e-12 * abs(tot_a[0]) * u0
    assert abs(tot_b[4] - tot_a[4]) <= 1e-11 * tot_a[4]
    assert abs(b[4] - a[4]) <= 1e-10 * a[4]


@pytest.mark.parametrize("lat,shape", [("D3Q27", (17, 9, 40)), ("D2Q9", (1, 17, 300))])
def test_chunk_length_changes_rounding_only(lbrr, gpu, monkeypatch, lat, shape):
    """Each node's moment sums are accumulated in the same order whatever the chunking (z-planes in
    3D, rows in 2D).  But the march is unrolled by 3 (register roles rotate with period 3), and in
    3D the planes next to a chunk go through code of their own, so a node is finalised in one of
    several copies of the iteration, depending on the chunk length; the compiler may fuse a
    multiply-add in one copy that it keeps apart in another.  Chunk lengths then agree to a few
    units in the last place (about 1e-9 on values of order 0.03), far below any indexing mistake."""
    rho, u, pi1 = TP.smooth_inputs(3 if shape[0] > 1 else 2, shape, 21)
    res = []
    for lz in ("1", "3", "17", "64"):
        monkeypatch.setenv("LBRR_MOM_LZ", lz)
        sim = lbrr.Simulation(lat, shape, 0.6, 4, storage="mom_fp32")
        sim.init_fields(rho, u, pi1)
        sim.step(5)
        res.append(sim.get_populations().cpu().numpy())
        sim.close()
    for lz, r in zip(("3", "17", "64"), res[1:]):
        d = float(np.abs(r - res[0]).max() / np.abs(res[0]).max())
        print(f"{lat} lz {lz} against lz 1: max rel diff {d:.1e}", flush=True)
        assert d <= 1e-6


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
def test_small_boxes_and_block_edges(lbrr, gpu, monkeypatch, lat):
    L = OL.lattice(lat)
    monkeypatch.setenv("LBRR_MOM_LZ", "2")
    if L.D == 2:
        # rows of 254 inner nodes per block, chunks of 2 rows here
        shapes = [(1, 1, 1), (1, 2, 1), (1, 1, 3), (1, 6, 30), (1, 7, 31), (1, 13, 61), (1, 3, 254), (1, 5, 255),
                  (1, 4, 509), (1, 9, 600)]
    else:
        # FP32 patches of 64 x 8 (inner 62 x 6), FP64 patches of 32 x 8 (inner 30 x 6)
        shapes = [(1, 1, 1), (1, 2, 3), (3, 1, 1), (2, 6, 30), (5, 7, 31), (3, 13, 61), (4, 5, 32), (2, 6, 62),
                  (5, 7, 63), (3, 12, 124), (4, 13, 125)]
    for k, shape in enumerate(shapes):
        print(f"edges {lat} shape={shape}", flush=True)
        ref = TP.oracle_run(lat, 4, 0.66, shape, 3, 500 + k)
        got = TP.gpu_run(lbrr, lat, 4, 0.66, shape, 3, 500 + k, "mom_fp64")
        e = errs(got, ref)
        assert e[0] <= 1e-12 and e[1] <= 1e-12 and e[2] <= 1e-10, (shape, e)
    if L.D == 3:
        # FP32 patches of 64 x 8 (inner 62 x 6): widths around one and two tiles, a tile
        # with a few target columns, a box narrower than the patch
        for k, shape in enumerate([(3, 5, 1), (2, 9, 2), (4, 7, 61), (3, 6, 62), (5, 7, 63), (2, 13, 64),
                                   (3, 7, 124), (2, 9, 126), (3, 30, 67), (2, 61, 70), (3, 200, 3)]):
            print(f"edges {lat} fp32 shape={shape}", flush=True)
            ref = TP.oracle_run(lat, 4, 0.66, shape, 3, 600 + k)
            got = TP.gpu_run(lbrr, lat, 4, 0.66, shape, 3, 600 + k, "mom_fp32")
            e = errs(got, ref)
            assert e[0] <= 1e-5 and e[1] <= 1e-5 and e[2] <= 1e-4, (shape, e)


def test_moment_storage_refuses_population_input_and_closure(lbrr, gpu):
    torch = gpu
    sim = lbrr.Simulation("D2Q9", (1, 8, 8), 0.6, 4, storage="mom_fp32")
    rho, u, pi1 = TP.smooth_inputs(2, (1, 8, 8), 3)
    sim.init_fields(rho, u, pi1)
    with pytest.raises(lbrr.LBError) as ei:
        sim.set_populations(torch.zeros((9, 1, 8, 8), dtype=torch.float32))
    assert ei.value.code == lbrr.LB_ERR_UNSUPPORTED
    params = torch.zeros(lbrr.LB_MLP_NPARAM, device="cuda", dtype=torch.float32)
    norm = torch.ones(lbrr.LB_MLP_NNORM, device="cuda", dtype=torch.float32)
    with pytest.raises(lbrr.LBError) as ei:
        sim.set_closure(params, norm)
    assert ei.value.code == lbrr.LB_ERR_UNSUPPORTED
    assert sim.bytes_per_update == 2 * 6 * 4
    sim.close()
