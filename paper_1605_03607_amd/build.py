"""Builds libhardspin.so (gfx950 kernels + C ABI) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhardspin.so")
PROBE_LIB = os.path.join(HERE, "libhsprobe.so")
SOURCES = ["hs_host.cpp", "hs_hardness.cpp", "hs_lao.cpp", "hs_pt.hip", "hs_gnn.hip", "hs_walk.hip", "hs_overlap.hip"]
ARCH = os.environ.get("HARDSPIN_ARCH", "gfx950")

# Packed FP32 instructions are disabled for every HIP translation unit.
HIP_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(hipcc, src, out_dir, verbose):
    obj = os.path.join(out_dir, src + ".o")
    cmd = [hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c",
           "-Wall", "-Wno-unused-result", *HIP_FLAGS, "-o", obj, os.path.join(CSRC, src)]
    if src.endswith(".cpp"):
        cmd.insert(1, "-x")
        cmd.insert(2, "hip")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def _link(hipcc, objs, lib, verbose):
    tmp = lib + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    _link(hipcc, [_compile(hipcc, "hs_probe.hip", out_dir, verbose)], PROBE_LIB, verbose)
    objs = []
    for src in SOURCES:
        objs.append(_compile(hipcc, src, out_dir, verbose))
    _link(hipcc, objs, LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
