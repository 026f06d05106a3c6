"""Compile the HIP library libh2.so in-tree for gfx950.

    python -m paper_2502_02395_amd.build_lib [--jobs N]

HIP sources are compiled with hipcc; the cluster-tree code is plain C++ built
with -ffp-contract=off so that the admissibility test follows the stated
operation order.  Objects go to csrc/_build/, the library next to this file.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libh2.so")
BUILD = os.path.join(CSRC, "_build")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_SOURCES = ["k_gemm.hip", "k_gemm_lp.hip", "k_gemm_f32.hip", "k_gemm_bf16.hip", "k_dense.hip", "k_vec.hip", "k_gather.hip", "mlp.hip"]
HOST_HIP_SOURCES = ["build.cpp", "solve.cpp", "gather_plan.cpp", "api.cpp"]
PLAIN_SOURCES = ["tree.cpp"]

# packed FP32 instructions are disabled: hand-checked FP32 paths only
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(line for line in r.stdout.splitlines() if "packed-fp32-ops" not in line
                    and "is not a recognized feature" not in line)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + out)
    return out


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cmds = []
    objs = []
    for s in HIP_SOURCES + HOST_HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in PLAIN_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-pthread", "-c",
                     os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread"] + objs + ["-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.v))
    sys.exit(0)
