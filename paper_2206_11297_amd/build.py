"""Build librsz.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librsz.so")
SOURCES = ["api.hip", "compress.hip", "decompress.hip"]

# -ffp-contract=off: no FMA contraction (the fp64 sums and the divide must be
# the plain IEEE operations); denormals preserved; packed fp32 disabled.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def build_lib(verbose=False, extra=()):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = ["hipcc", *FLAGS, *extra, "-o", LIB + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build_lib(verbose=True))
