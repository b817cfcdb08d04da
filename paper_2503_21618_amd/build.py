"""Builds libslrf.so (gfx950) in-tree: host C++ with g++, HIP sources with hipcc.

    python -m paper_2503_21618_amd.build        (or build() from Python)
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libslrf.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HOST_SRC = ["dense.cpp", "poles.cpp"]
HIP_SRC = ["kernels.hip", "krylov.hip", "solver.hip"]
# packed FP32 instructions are disabled for all device code
HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} {cmd[-1]}")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    steps = []
    for src in HOST_SRC:
        obj = os.path.join(BUILD, src + ".o")
        steps.append((["g++", "-O3", "-fPIC", "-std=c++17", "-pthread", "-c", os.path.join(CSRC, src),
                       "-o", obj], obj))
    for src in HIP_SRC:
        obj = os.path.join(BUILD, src + ".o")
        steps.append(([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(steps), 4)) as pool:
        list(pool.map(lambda st: _run(st[0]), steps))
    objs = [obj for _, obj in steps]
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
