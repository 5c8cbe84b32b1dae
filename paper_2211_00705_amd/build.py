"""Builds the HIP library libimexds.so for gfx950 (in-tree, next to this file)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libimexds.so")
SOURCES = [os.path.join(HERE, "csrc", "imexds_kernels.hip"),
           os.path.join(HERE, "csrc", "imexds_zone8.hip"),
           os.path.join(HERE, "csrc", "imexds_zpair.hip"),
           os.path.join(HERE, "csrc", "imexds_znewton.hip"),
           os.path.join(HERE, "csrc", "imexds_adjoint.hip"),
           os.path.join(HERE, "csrc", "imexds_runtime.hip"),
           os.path.join(HERE, "csrc", "euler.hip"),
           os.path.join(HERE, "csrc", "creation.hip"),
           os.path.join(HERE, "csrc", "ctube.hip")]
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
         # IEEE FP64 evaluated as written: no fused multiply-add contraction
         "-ffp-contract=off",
         # keep hipcc from emitting packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False):
    """Compiles the library (always recompiles) and returns its path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
