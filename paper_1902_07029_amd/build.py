"""Build the lsmg HIP library for gfx950 in-tree (``liblsmg.so`` next to this file).

Six translation units: ``build.hip`` (hierarchy construction, compiled with
FMA contraction off so the discrete geometry is evaluated in plain IEEE order),
``kernels.hip`` (V-cycle and Newton kernels), ``tail.hip`` (the coarse tail held
in LDS and its tables), ``init.hip`` (level-set preparation, FMA contraction
off), ``api.hip`` (the C ABI and the single-hierarchy drivers) and ``batch.hip``
(batches of hierarchies).  Every HIP compile line disables packed FP32
instructions.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "liblsmg.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")

ARCH = os.environ.get("LSMG_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", CSRC, "-I", INCLUDE,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
UNITS = [("build.hip", ["-ffp-contract=off"]), ("kernels.hip", []), ("tail.hip", []), ("init.hip", ["-ffp-contract=off"]),
         ("api.hip", []),
         ("batch.hip", [])]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    objs = []
    for src, extra in UNITS:
        obj = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
        cmd = [cc, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + extra
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fPIC"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
