"""Builds libscasm.so in-tree with hipcc for gfx950.

    python -m paper_2509_21037_amd.build
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libscasm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-march=x86-64-v3"]
DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
                # packed FP32 vector ops stay off (hipcc's host pass warns it
                # does not know the feature; harmless)
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for src, kind in (("planner.cpp", "host"), ("dense_host.cpp", "host"), ("scasm.cpp", "hosthip"), ("kernels.hip", "device"),
                      ("apply.hip", "device")):
        obj = os.path.join(BUILD, src + ".o")
        path = os.path.join(CSRC, src)
        if kind == "host":
            cmd = [HIPCC, *HOST_FLAGS, "-x", "c++", *inc, "-c", path, "-o", obj]
        elif kind == "hosthip":
            cmd = [HIPCC, *HOST_FLAGS, "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-x", "c++", *inc, "-c", path, "-o", obj]
        else:
            cmd = [HIPCC, *DEVICE_FLAGS, *inc, "-c", path, "-o", obj]
        _run(cmd, verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fopenmp", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
