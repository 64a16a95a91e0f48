"""Build the HIP library (gfx950) in-tree: paper_1912_13132_amd/libpcv.so.

Every call compiles from source.  Kernels (.hip) are compiled for gfx950
only, with packed FP32 instructions disabled; host sources (.cpp) are
compiled as plain C++ against the HIP runtime headers.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libpcv.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HIP_SOURCES = ["pcv_potrf.hip", "pcv_kernels.hip", "pcv_krige.hip", "pcv_partition.hip", "pcv_noalloc.hip"]
CPP_SOURCES = ["pcv_capi.cpp", "pcv_problem.cpp", "pcv_server.cpp", "pcv_tune.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
DEVICE = ["-x", "hip", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
HOST = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(ln for ln in r.stdout.splitlines() if "packed-fp32-ops" not in ln)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)
    return out


def build(verbose=False, jobs=4):
    os.makedirs(OBJ, exist_ok=True)
    cmds = []
    objs = []
    for src in HIP_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        cmds.append([HIPCC] + COMMON + DEVICE + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for src in CPP_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        cmds.append([HIPCC] + COMMON + HOST + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
         + ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lpthread", "-Wl,-rpath," + os.path.join(ROCM, "lib")],
         verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
