"""Builds ``librlb.so`` (HIP for gfx950) in-tree with hipcc.

Packed FP32 instructions are disabled for all device code
(``-packed-fp32-ops``); the host pass warns that it does not know the target
feature, which is harmless.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librlb.so")
SOURCES = ["rlb_kernels.hip", "rlb_adjoint.hip", "rlb_feq.hip", "rlb_plane.hip", "rlb_box.hip", "rlb_noalloc.hip",
           "rlb_api.cpp", "rlb_plane_api.cpp", "rlb_box_api.cpp", "quadrature.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra=()) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wall", "-Wno-unused-function", *extra]
    procs = []
    for src in SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc(), *common, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    for p, src in procs:
        _, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(err)
            raise RuntimeError(f"hipcc failed on {src}")
        elif verbose and err.strip():
            sys.stderr.write("".join(l + "\n" for l in err.splitlines() if "packed-fp32-ops" not in l))
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
