"""Build the HIP library libmhd.so for gfx950 (in-tree).

hipcc compiles the kernels and the C-ABI host code in one shared library.
Floating-point contraction is limited to single expressions
(-ffp-contract=on) so that a value recomputed by two blocks from the same
inputs rounds identically; packed FP32 instructions are disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmhd.so")
SOURCES = ["mhd_api.hip", "mhd_kernels.hip", "mhd_diffusion.hip", "mhd_flatten.hip",
           "mhd_species.hip", "mhd_mathcheck.hip", "mhd_noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -amdgpu-mfma-vgpr-form: the matrix instructions of the guess network
# write their results to ordinary VGPRs, so the vector work that packs them
# for the next layer reads them directly instead of copying each value out
# of the accumulation registers first (the kernels without matrix
# instructions are unaffected).
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False, extra=None) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [HIPCC] + FLAGS + list(extra or []) + srcs + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
