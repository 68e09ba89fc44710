"""Builds the gfx950 HIP library libpinnjet.so in-tree.

Every source under csrc/ is compiled by hipcc for gfx950 only, in parallel,
then linked into one shared library next to this file.  Packed FP32 VALU
instructions are disabled for all device code.  Except in the k_layer
sources (where it measured slower), MFMA instructions are selected in their VGPR form
(accumulators in ordinary VGPRs), which keeps the compiler from shuffling
loop-carried accumulators through AGPRs.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpinnjet.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=on: a*b + c is fused into one FMA only within a single source
# expression, never across statements.  Kernels that inline the same device
# code (the direct and grouped launches of a body, the stored-state and
# recompute variants of the backward) then round identically, which the
# bitwise checkpoint, graph and ensemble equalities rely on.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


MFMA_VGPR = ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
NO_MFMA_VGPR_PREFIX = "k_layer"


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    extra = [] if os.path.basename(src).startswith(NO_MFMA_VGPR_PREFIX) else MFMA_VGPR
    cmd = [HIPCC] + FLAGS + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, jobs=int(sys.argv[1]) if len(sys.argv) > 1 else 8)
