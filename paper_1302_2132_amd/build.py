"""Build libgks.so (HIP, gfx950) in-tree."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgks.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled (-packed-fp32-ops): some of their forms have given
# wrong results on this hardware; the compiler then emits scalar FP32 instead.
# Machine-level loop-invariant code motion is disabled: in the grid-stride face kernels it
# hoists every FP64 constant of the flux (polynomial coefficients of exp and of the
# time-weight series) out of the tile loop into VGPRs, which cost the 2D FP64 kernel ~60
# VGPRs (236 instead of 175, so 2 waves per SIMD instead of 3) and made the 3D FP64
# kernel spill.  Without it the constants are materialised in SGPRs next to their use.
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-disable-machine-licm",
         "-Wall", "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    src = os.path.join(CSRC, "gks_lib.hip")
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp, src]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libgks.so")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
