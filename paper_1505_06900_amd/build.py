"""Build the HIP library liblbrr.so in-tree for gfx950 (hipcc, no GPU needed).

Usage: python -m paper_1505_06900_amd.build [-j JOBS] [--verbose]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "liblbrr.so")
# per-kernel register, scratch, LDS and occupancy figures reported by the compiler
RESOURCES = os.path.join(PKG, "liblbrr_resources.json")

SOURCES = ["api.hip", "diag.hip", "probe.hip", "closure.hip", "kernels_d2q9.hip", "kernels_d3q19.hip", "kernels_d3q27.hip"]

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=fast",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # per-kernel resource usage as compiler remarks (analysis only; collected into RESOURCES)
    "-Rpass-analysis=kernel-resource-usage",
]

# per-source additions: the closure kernels take matrix-core results in ordinary
# VGPRs, so the activations read them without a copy from the accumulation registers
SOURCE_FLAGS = {"closure.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def parse_resource_remarks(text):
    """{kernel name: {field: value}} from the compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        if "remark:" not in line or "kernel-resource-usage" not in line:
            continue
        body = line.split("remark:", 1)[1].rsplit("[-Rpass-analysis", 1)[0].strip()
        key, _, val = body.partition(":")
        key, val = key.strip(), val.strip()
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None and val:
            cur[key] = int(val) if val.lstrip("-").isdigit() else val
    return out


def demangle(names):
    exe = shutil.which("c++filt") or shutil.which("llvm-cxxfilt")
    if not exe or not names:
        return {n: n for n in names}
    r = subprocess.run([exe], input="\n".join(names), capture_output=True, text=True)
    out = r.stdout.splitlines() if r.returncode == 0 else []
    return dict(zip(names, out)) if len(out) == len(names) else {n: n for n in names}


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found (ROCm toolchain required to build liblbrr.so)")
    return exe


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, *SOURCE_FLAGS.get(src, []), "-I", os.path.join(ROOT, "include"), "-c",
           os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(jobs=None, verbose=False):
    """Compile every source and link liblbrr.so.  Always recompiles."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    res = {}
    for _, err in results:
        res.update(parse_resource_remarks(err))
    names = demangle(sorted(res))
    with open(RESOURCES, "w") as fh:
        json.dump({names[k]: v for k, v in sorted(res.items())}, fh, indent=1)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose))


if __name__ == "__main__":
    sys.exit(main())
