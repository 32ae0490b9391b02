"""Build libgks.so (HIP, gfx950) in-tree.

The library is one host unit (gks_lib.hip: the C ABI and the small kernels) plus the
face-kernel instantiations of gks_inst.hip, compiled once per share (GKS_PART 0..7).  The
units compile in parallel into paper_1302_2132_amd/_build/ and are linked into libgks.so.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgks.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
NPARTS = 8

# Packed FP32 instructions are disabled (-packed-fp32-ops): some of their forms have given
# wrong results on this hardware; the compiler then emits scalar FP32 instead.
# Machine-level loop-invariant code motion is disabled: in the grid-stride face kernels it
# hoists every FP64 constant of the flux (polynomial coefficients of exp and of the
# time-weight series) out of the tile loop into VGPRs, which cost the 2D FP64 kernel ~60
# VGPRs (236 instead of 175, so 2 waves per SIMD instead of 3) and made the 3D FP64
# kernel spill.  Without it the constants are materialised in SGPRs next to their use.
CFLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-disable-machine-licm",
          "-Wall", "-Wno-unused-command-line-argument"]
FLAGS = CFLAGS + ["-shared"]     # single-command form (one source to a shared object)


def units():
    """(source, extra flags, object name) of every compilation unit."""
    out = [(os.path.join(CSRC, "gks_lib.hip"), [], "gks_lib.o")]
    for p in range(NPARTS):
        out.append((os.path.join(CSRC, "gks_inst.hip"), [f"-DGKS_PART={p}"], f"gks_inst_{p}.o"))
    return out


def compile_unit(src, extra, obj, more=()):
    cmd = [HIPCC] + CFLAGS + list(extra) + list(more) + ["-c", "-o", obj, src]
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(units()), os.cpu_count() or 1, 16)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = []
        for src, extra, name in units():
            obj = os.path.join(OBJ, name)
            objs.append(obj)
            futs.append((name, ex.submit(compile_unit, src, extra, obj + ".tmp")))
        failed = False
        for name, f in futs:
            r = f.result()
            if r.returncode != 0:
                sys.stderr.write(f"--- {name}\n" + r.stdout + r.stderr)
                failed = True
            elif verbose:
                sys.stderr.write(r.stderr)
        if failed:
            raise RuntimeError("hipcc failed building libgks.so")
    for obj in objs:
        os.replace(obj + ".tmp", obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking libgks.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
