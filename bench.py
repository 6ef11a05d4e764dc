"""Benchmark: D3Q27 recursive-regularised stream+collide, 256^3 periodic 3D
Taylor--Green vortex (Ma 0.1, Re 1600, order 4), on one MI355X.

Prints ONE JSON line.  ``value`` is the throughput in GLUPS (10^9 lattice-node
updates per second) of FP32 population storage, inputs resident in HBM.  The
same line carries the FP16-deviation and FP64 storage rates, the L2 velocity
error of each storage against the FP64 storage run after the workload's
10,000 steps, run apart from the timed region (FP64 mode is itself
parity-checked against the oracle), the
HBM roofline of the step kernel (algorithmic bytes 2*q*s per node over the
HIP-event-timed average launch) and the FP64 CPU oracle timed on a bounded
sample of the same workload.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
STORAGE_NAMES = {"fp32": "FP32 population storage", "fp16": "FP16 population storage",
                 "fp64": "FP64 population storage", "mom_fp32": "FP32 moment storage",
                 "mom_fp64": "FP64 moment storage"}
METRIC = "GLUPS + % HBM peak, D3Q27 RR-BGK 256³ FP32 vs FP16-store; L2 err vs FP64"
WORKLOAD = "tgv3d_256_ma01"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_step_d3q27_o4_256.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Sources of the D3Q27 step kernels: the counters stay valid while these are unchanged.
STEP_SOURCES = ("lattice.hpp", "collide.hpp", "ops.hpp", "kernels.hpp", "mkernels.hpp", "ops_impl.hpp",
                "kernels_d3q27.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1505_06900_amd", "csrc")
    for name in STEP_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(storage):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it matches this source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    ent = d.get(storage)
    return None if ent is None else ent.get("bytes_per_launch")


def run_gpu(P, torch, storage, rho, u, cfg, steps, warmup, repeats=0, repeat_steps=200):
    """Warm up, then time ``steps`` steps (wall clock and HIP events on the library's stream).
    With repeats > 0, after the timed region: ``repeats`` more event-timed runs of
    ``repeat_steps`` steps each, reported as kernel-time GLUPS (median, min, max)."""
    n = cfg["n"]
    sim = P.Simulation("D3Q27", (n, n, n), cfg["tau"], cfg["order"], storage=storage)
    sim.init_fields(rho, u)
    sim.step(warmup)
    stream = sim.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    nodes = n**3
    res = {
        "glups": nodes * steps / wall / 1e9,
        "ms_per_step": wall * 1e3 / steps,
        "kernel_ms": ev_ms / steps,
        "bytes_per_update": sim.bytes_per_update,
    }
    totals = sim.reduce()
    if repeats > 0:
        rates = []
        for _ in range(repeats):
            e0.record(stream)
            sim.step(repeat_steps)
            e1.record(stream)
            torch.cuda.synchronize()
            rates.append(nodes * repeat_steps / (e0.elapsed_time(e1) * 1e-3) / 1e9)
        rates.sort()
        res["repeats"] = {"runs": repeats, "steps": repeat_steps, "median_glups": round(rates[len(rates) // 2], 3),
                          "min_glups": round(rates[0], 3), "max_glups": round(rates[-1], 3)}
    sim.close()
    return res, totals


def horizon_errors(P, torch, storages, rho, u, cfg, steps):
    """Relative L2 error of u after ``steps`` steps (the workload's own step count, independent of
    the timed region) of each storage against the FP64 population run from the same fields; the
    FP64 mode is itself held to the oracle at 1e-12."""
    n = cfg["n"]

    def final_u(storage):
        sim = P.Simulation("D3Q27", (n, n, n), cfg["tau"], cfg["order"], storage=storage)
        sim.init_fields(rho, u)
        sim.step(steps)
        _, vel = sim.moments()
        sim.close()
        return vel

    ref = final_u("fp64")
    out = {"steps": steps, "reference": "fp64"}
    for st in storages:
        if st != "fp64":
            v = final_u(st)
            out[st] = float(f"{float(torch.linalg.vector_norm(v - ref) / torch.linalg.vector_norm(ref)):.3e}")
            del v
    return out


def device_record(torch):
    """The device and software the numbers were taken on: GPU, ROCm / HIP / torch versions,
    current clocks and power limits as rocm-smi reports them (None where unavailable)."""
    import subprocess

    props = torch.cuda.get_device_properties(0)
    rec = {"name": props.name, "arch": getattr(props, "gcnArchName", None), "compute_units": props.multi_processor_count,
           "hbm_gib": round(props.total_memory / 2**30, 1), "hip_runtime": torch.version.hip, "torch": torch.__version__}
    try:
        with open("/opt/rocm/.info/version") as fh:
            rec["rocm"] = fh.read().strip()
    except OSError:
        rec["rocm"] = None
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--showmaxpower", "--showpower", "--json"],
                           capture_output=True, text=True, timeout=30)
        card = next(iter(json.loads(r.stdout).values())) if r.returncode == 0 else {}
        rec["smi"] = {k: v for k, v in card.items() if "clock" in k.lower() or "power" in k.lower()
                      or k.lower().startswith(("sclk", "mclk", "fclk"))}
    except (OSError, ValueError, StopIteration, subprocess.TimeoutExpired):
        rec["smi"] = None
    return rec


def kernel_resources(B, storage):
    """Registers, scratch, LDS and occupancy of the D3Q27 order-4 step kernel of ``storage``, as the
    compiler reported them when the library was built."""
    name = {"fp32": "k_step<lbrr::D3Q27, 4, float>", "fp16": "k_stepINS_5D3Q27ELi4EDF16_",
            "fp64": "k_step<lbrr::D3Q27, 4, double>", "mom_fp32": "k_mstep_t<lbrr::D3Q27, 4, float, 9, false>",
            "mom_fp64": "k_mstep<lbrr::D3Q27, 4, double, 8, 32, false>"}[storage]
    try:
        with open(B.RESOURCES) as fh:
            res = json.load(fh)
    except (OSError, ValueError):
        return None
    for k, v in res.items():
        if name in k:
            return {"kernel": k, **v}
    return None


def copy_probe(P, torch, nbytes=2 << 30, reps=10):
    """Achievable HBM rate of a plain device copy (read n + write n bytes) with the library's copy kernel."""
    import ctypes

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    P.check(P.lb_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes, sp))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        P.check(P.lb_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes, sp))
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"bytes_moved_per_launch": 2 * nbytes, "ms": round(ms, 4), "gbs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def probe_table(P, torch, nbytes=2 << 30, reps=10):
    """HBM rates of plain access patterns (lb_probe_bandwidth) on 2 GiB buffers: copy, read, write
    and the copy of q equal planes, by bytes per lane, one-shot or persistent grid, plain or
    non-temporal accesses.  GB/s counts the bytes each launch reads plus those it writes."""
    import ctypes

    src = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    names = {0: "copy", 1: "read", 2: "write", 3: "stream copy"}
    configs = []
    for kind in (0, 1, 2):
        for vec in (4, 8, 16):
            for bpc in (0, 2, 4, 8, 16):
                for nt in (0, 1):
                    configs.append((kind, vec, bpc, nt, 1))
    for streams in (1, 2, 4, 9, 18, 27, 32):
        for vec in (4, 8, 16):
            for nt in (0, 1):
                configs.append((3, vec, 0, nt, streams))
    rows = []
    for kind, vec, bpc, nt, streams in configs:
        n = nbytes - nbytes % (16 * streams * vec) if kind == 3 else nbytes
        args = (kind, vec, bpc, nt, streams, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n, sp)
        P.check(P.lb_probe_bandwidth(*args))
        P.check(P.lb_probe_bandwidth(*args))
        e0.record(stream)
        for _ in range(reps):
            P.check(P.lb_probe_bandwidth(*args))
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        moved = n * (2 if kind in (0, 3) else 1)
        rows.append({"kind": names[kind], "vec_bytes": vec, "blocks_per_cu": bpc, "nontemporal": nt,
                     "streams": streams, "bytes": moved, "ms": round(ms, 4),
                     "gbs": round(moved / (ms * 1e-3) / 1e9, 1)})
        log(f"probe {rows[-1]}")
    del src, dst
    return rows


def probe(P, torch, storages, steps=5, lattices=(("D3Q27", None),)):
    """Short fixed launch sequence for hardware-counter runs: copies of known size, then step kernels
    (each lattice and order of ``lattices``, order None = the workload's, every storage)."""
    import ctypes

    import workloads as W

    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(3):
        P.check(P.lb_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes, sp))
    torch.cuda.synchronize()
    del src, dst
    cfg = W.WORKLOADS[WORKLOAD]
    n = cfg["n"]
    rho, u = W.tgv3d(n, cfg["u0"])
    for lat, order in lattices:
        order = order or cfg["order"]
        for st in storages:
            sim = P.Simulation(lat, (n, n, n), cfg["tau"], order, storage=st)
            sim.init_fields(rho, u)
            sim.step(steps)
            torch.cuda.synchronize()
            log(f"probe {lat} order {order} {st}: {steps} steps, "
                f"{sim.bytes_per_update * n**3:.0f} algorithmic bytes per launch")
            sim.close()
    return {"copy_bytes": nbytes, "copies": 3, "storages": storages, "steps": steps, "nodes": n**3,
            "lattices": [f"{lat}:{order or cfg['order']}" for lat, order in lattices]}


def summarize_prof(paths):
    """Text summary of rocprofv3 CSV output: kernel_stats (durations) and counter_collection (PMC)."""
    import csv
    import glob

    lines = []
    for root in paths:
        for f in sorted(glob.glob(os.path.join(root, "**", "*kernel_stats.csv"), recursive=True)):
            lines.append(f"# kernel stats: {os.path.relpath(f, root)}")
            with open(f) as fh:
                rows = list(csv.DictReader(fh))
            for r in rows:
                lines.append(f"{r['Name'][:90]:90s} calls {r['Calls']:>6s} avg_us {float(r['AverageNs'])/1e3:10.2f} "
                             f"min_us {float(r['MinNs'])/1e3:10.2f} max_us {float(r['MaxNs'])/1e3:10.2f}")
        for f in sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True)):
            lines.append(f"# counters: {os.path.relpath(f, root)}")
            acc = {}
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    key = (r["Kernel_Name"][:90], r["Counter_Name"])
                    acc.setdefault(key, []).append(float(r["Counter_Value"]))
            for (k, c), v in sorted(acc.items()):
                lines.append(f"{k:90s} {c:12s} dispatches {len(v):4d} mean {sum(v)/len(v):16.1f} "
                             f"min {min(v):16.1f} max {max(v):16.1f}")
    return "\n".join(lines)


def closure_run(log_fn=None):
    """Learned a1^(2) closure on decaying 2D turbulence (fine 1024^2, coarse 256^2, D2Q9 order 4).

    Trains on seeds 0-3 with the library's kernels and compares the closure run with the plain
    coarse run against the coarse-grained fine run (held-out seed 4, 2000 coarse steps)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1505_06900_amd import closure as C

    cf, cc = dict(W.WORKLOADS["turb2d_fine_1024"]), dict(W.WORKLOADS["turb2d_coarse_256"])
    t0 = time.perf_counter()
    xs, ys = [], []
    for seed in range(4):
        x, y = C.generate(seed, cf, cc, snapshots=40, interval=200)
        xs.append(x)
        ys.append(y)
    x, y = torch.cat(xs), torch.cat(ys)
    del xs, ys
    xt, yt = C.generate(4, cf, cc, snapshots=20, interval=200)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    norm = C.norm_stats(x, y)
    t0 = time.perf_counter()
    steps, batch = 3000, 4096
    params, losses = C.train(x, y, norm, steps=steps, batch=batch, lr=1e-3, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    r2 = C.r2_score(C.predict(params, norm, xt), yt)
    res = C.a_posteriori(params, norm, 4, cf, cc, coarse_steps=2000, every=200)
    ep, ec = res["err_u"]["plain"], res["err_u"]["closure"]
    return {
        "workload": "decaying 2D turbulence, D2Q9 order 4, fine 1024^2 tau 0.535472, coarse 256^2 tau 0.508868",
        "train_samples": int(x.shape[0]), "train_steps": steps, "batch": batch,
        "train_s": round(t_train, 2), "datagen_s": round(t_gen, 2),
        "mlp_train_tflops": round(6 * 6723 * batch * steps / t_train / 1e12, 3),
        "final_loss": round(losses[-1][1], 5), "heldout_r2": [round(float(v), 4) for v in r2],
        "u_err_vs_filtered_fine_at_2000": {"plain": round(ep[-1], 5), "closure": round(ec[-1], 5)},
        "stable": res["stable"], "step_ms": {k: round(v, 4) for k, v in res["step_ms"].items()},
        "cost_ratio": round(res.get("cost_ratio", float("nan")), 2),
    }


def write_traffic(fetch_dir, write_dir, out_path):
    """HBM bytes per launch of the step kernels from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of --probe.

    Counters are in KiB per dispatch; each is scaled by what it reads for the
    probe's plain copy of known size (1 GiB read + 1 GiB written).
    """
    import csv
    import glob

    def load(d, counter):
        acc = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] == counter:
                        acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy_kib = (1 << 30) / 1024.0
    kf = [k for k in fetch if "k_copy" in k][0]
    ff, fw = copy_kib / fetch[kf], copy_kib / write[kf]
    nodes = 256**3
    out = {"source_hash": kernel_source_hash(), "copy_calibration": {"fetch_factor": ff, "write_factor": fw},
           "workload": "D3Q27 order 4, 256^3, one step launch"}
    tags = {"fp32": ("k_step", "float"), "fp16": ("k_step", "DF16_"), "fp64": ("k_step", "double"),
            "mom_fp32": ("k_mstep", "float"), "mom_fp64": ("k_mstep", "double")}
    for st, (kern, tag) in tags.items():
        ks = [k for k in fetch if kern in k and "D3Q27" in k and tag in k and "4" in k]
        if not ks:
            continue
        k = ks[0]
        b = (fetch[k] * ff + write[k] * fw) * 1024.0
        alg = {"fp32": 216, "fp16": 108, "fp64": 432, "mom_fp32": 80, "mom_fp64": 160}[st] * nodes
        out[st] = {"kernel": k, "fetch_kib": fetch[k], "write_kib": write[k], "bytes_per_launch": round(b),
                   "algorithmic_bytes": alg, "ratio": round(b / alg, 5)}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def host_threads():
    """Threads the host may use: OMP_NUM_THREADS when set (the share of a shared machine), else
    the CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_baseline(cfg, budget_s=10.0):
    """The FP64 oracle on a 32^3 box of the same flow (same Re, Ma), timed with the host's
    threads (numpy's BLAS pool) and with one thread, about ``budget_s`` seconds each."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    import workloads as W
    from oracle import lattice as OL
    from oracle import rr

    n = 32
    L = OL.lattice("D3Q27")
    tau = 0.5 + 3 * (cfg["u0"] * (n / (2 * math.pi)) / 1600.0)  # same Re at the smaller box
    rho, u = W.tgv3d(n, cfg["u0"])

    def timed(threads):
        f = rr.init_populations(L, cfg["order"], rho, u)
        steps = 0
        with threadpool_limits(threads):
            used = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < budget_s:
                f = rr.step(L, cfg["order"], tau, f)
                steps += 1
            dt = time.perf_counter() - t0
        assert np.isfinite(f).all()
        return n**3 * steps / dt / 1e9, steps, dt, used

    v_all, s_all, dt_all, used = timed(host_threads())
    v_one, s_one, dt_one, _ = timed(1)
    return {
        "value": v_all,
        "unit": "GLUPS",
        "cores": used,
        "kind": "oracle",
        "sample": f"D3Q27 order {cfg['order']} TGV at 32^3 (same Re and Ma), FP64 numpy: {s_all} steps in "
                  f"{dt_all:.1f} s with {used} BLAS threads; {s_one} steps in {dt_one:.1f} s with 1 thread",
        "single_thread_value": v_one,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--horizon", type=int, default=None,
                    help="steps of the velocity-error runs against FP64 (default: the workload's 10000)")
    ap.add_argument("--no-closure", action="store_true", help="skip the learned-closure measurement")
    ap.add_argument("--storages", default="fp32,fp16,fp64,mom_fp32",
                    help="state storages to time; the first one is the headline value")
    ap.add_argument("--probe", action="store_true", help="short launch sequence for rocprofv3 counter runs")
    ap.add_argument("--probe-lattices", default="D3Q27:4",
                    help="lattice:order list of the --probe step kernels (3D lattices, 256^3 Taylor-Green fields)")
    ap.add_argument("--probe-table", action="store_true", help="HBM rates of plain access patterns, then exit")
    ap.add_argument("--summarize-prof", nargs="+", metavar="DIR", help="summarise rocprofv3 CSV output and exit")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the HBM traffic summary of the step kernels from two --pmc runs of --probe")
    a = ap.parse_args(argv)
    if a.summarize_prof:
        print(summarize_prof(a.summarize_prof))
        return 0
    if a.write_traffic:
        print(json.dumps(write_traffic(*a.write_traffic, TRAFFIC_FILE), indent=1))
        return 0
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the step would shard by z-slabs with a halo exchange per step, not implemented); use --gpus 1",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1505_06900_amd import build as B

    if not os.path.exists(B.LIB):
        B.build()
    import paper_1505_06900_amd as P
    import workloads as W

    if a.probe:
        lats = []
        for spec in a.probe_lattices.split(","):
            lat, _, order = spec.partition(":")
            if lat not in ("D3Q19", "D3Q27") or not order.isdigit():
                print(f"bad --probe-lattices entry {spec!r} (want D3Q19:N or D3Q27:N)", file=sys.stderr)
                return 2
            lats.append((lat, int(order)))
        print(json.dumps(probe(P, torch, a.storages.split(","), lattices=lats)), flush=True)
        return 0
    if a.probe_table:
        print(json.dumps(probe_table(P, torch)), flush=True)
        return 0
    cfg = W.WORKLOADS[WORKLOAD]
    n = cfg["n"]
    log(f"generating {n}^3 TGV fields")
    rho, u = W.tgv3d(n, cfg["u0"])
    rho_t = torch.from_numpy(rho).cuda()
    u_t = torch.from_numpy(u).cuda()
    del rho, u
    storages = a.storages.split(",")
    results = {}
    for st in storages:
        log(f"running {st}: warmup {a.warmup}, timed {a.steps}")
        res, totals = run_gpu(P, torch, st, rho_t, u_t, cfg, a.steps, a.warmup,
                              repeats=5 if st == storages[0] else 0)
        results[st] = res
        log(f"{st}: {res['glups']:.2f} GLUPS, kernel {res['kernel_ms']:.3f} ms, totals {totals[0]:.6e}")
    horizon = a.horizon if a.horizon is not None else cfg["steps"]
    log(f"velocity error of each storage against FP64 after {horizon} steps")
    errs = horizon_errors(P, torch, storages, rho_t, u_t, cfg, horizon)
    log(f"errors: {errs}")
    main_st = storages[0]
    r = results[main_st]
    nodes = n**3
    achieved = r["bytes_per_update"] * nodes / (r["kernel_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(main_st)
    out = {
        "metric": METRIC,
        "value": round(r["glups"], 3),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f32 (f16 storage)", "fp64": "f64", "mom_fp32": "f32 (moment storage)",
                  "mom_fp64": "f64 (moment storage)"}[main_st],
        "data": "synthetic",
        "config": {"workload": "3D Taylor-Green vortex 256^3 periodic, D3Q27 order 4, Ma 0.1, Re 1600, "
                               f"tau {cfg['tau']}, {STORAGE_NAMES[main_st]}",
                   "lattice": "D3Q27", "order": cfg["order"], "nodes": nodes, "storage": main_st},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "storage_rates": {st: {"glups": round(v["glups"], 3), "kernel_ms": round(v["kernel_ms"], 4),
                               "hbm_frac": round(v["bytes_per_update"] * nodes / (v["kernel_ms"] * 1e-3) / 1e12
                                                 / (HBM_PEAK_GBS / 1000), 4),
                               "bytes_per_update": v["bytes_per_update"]} for st, v in results.items()},
        "l2_err_u_vs_fp64": errs,
        "repeats": r.get("repeats"),
        "kernel_resources": kernel_resources(B, main_st),
        "device": device_record(torch),
    }
    out["copy_probe"] = copy_probe(P, torch)
    log(f"copy probe: {out['copy_probe']['gbs']} GB/s")
    if not a.no_closure:
        log("learned closure: data generation, training, a-posteriori comparison")
        out["closure"] = closure_run()
        log(f"closure: {out['closure']['u_err_vs_filtered_fine_at_2000']}")
    if not a.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
