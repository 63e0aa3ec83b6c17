"""Build librmx.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2104_00095_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librmx.so")
SOURCES = ["rmx_kernels.hip", "rmx_step.hip", "rmx_blur.hip", "rmx_plan.cpp", "rmx_core.cpp",
           "rmx_server.cpp"]
# Per-file flags: the time-step and blur-zone kernels evaluate their arithmetic in the
# written order.
EXTRA = {"rmx_step.hip": ["-ffp-contract=off"], "rmx_blur.hip": ["-ffp-contract=off"]}
# No packed-FP32 instructions; device code for gfx950 only.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc"] + HIPFLAGS + EXTRA.get(src, []) + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                      "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd.insert(1, "-xhip")
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
