"""Build ``libtartarus.so`` (HIP kernels + C-ABI runtime) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtartarus.so")
SOURCES = ["trace_kernel.hip", "aux_kernels.hip", "noalloc.hip", "runtime.cpp", "host_logic.cpp"]
ARCH = "gfx950"

# Packed FP32 instructions stay disabled (-packed-fp32-ops): some of their forms
# have given silently wrong results on these machines.
# -disable-machine-licm: FP64 VALU instructions cannot encode 64-bit literals,
# so every FP64 constant (Runge-Kutta tableau, polynomial coefficients) is
# materialised in a VGPR pair; hoisting them all out of the persistent loop
# costs ~60 VGPRs and forces scratch spills.  Rematerialising them at the use
# keeps the integrator spill-free.
# -fmacf64-inst: without the two-address v_fmac_f64 the compiler emits the
# three-address v_fma_f64, which takes a scalar-register addend directly; with
# it, every fused multiply-add whose addend is a coefficient in scalar
# registers first copied that coefficient into a VGPR pair (two moves).
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Xclang", "-target-feature", "-Xclang", "-fmacf64-inst",
    "-mllvm", "-disable-machine-licm",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def resource_usage(src: str = "trace_kernel.hip") -> str:
    """Compiler's per-kernel register / occupancy report for a source file."""
    cmd = [hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return r.stderr


if __name__ == "__main__":
    build(verbose=True)
    if "--usage" in sys.argv:
        print(resource_usage())
