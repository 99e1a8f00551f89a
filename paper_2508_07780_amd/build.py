"""Build the HIP C-ABI library (gfx950) in-tree: paper_2508_07780_amd/libddfem.so."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libddfem.so")
SOURCES = ["kernels.hip", "cga.hip", "paper_grad.hip", "initial.hip", "mesh.cpp", "api.cpp"]
ARCH = os.environ.get("DD_OFFLOAD_ARCH", "gfx950")


def hipcc_command(out=LIB, defines=()):
    return [
        "hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        *[f"-D{d}" for d in defines],
        # packed FP32 instructions are disabled for all device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        *[os.path.join(CSRC, s) for s in SOURCES],
        "-o", out,
    ]


def build(verbose=True, out=LIB, defines=()):
    tmp = out + ".tmp"
    cmd = hipcc_command(tmp, defines)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    # optional: OUT_PATH DEFINE...  (e.g. a tile-shape variant for a comparison run)
    if len(sys.argv) > 1:
        build(out=os.path.abspath(sys.argv[1]), defines=sys.argv[2:])
    else:
        build()
    sys.exit(0)
