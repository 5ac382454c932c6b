"""Build the gfx950 shared library libstucker.so in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with packed FP32 instructions
disabled, then linked with rocSOLVER/rocBLAS (used for the small FP64
symmetric eigendecompositions).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libstucker.so")
SOURCES = ["k_fiber_ff.hip", "k_fiber_fd.hip", "k_fiber_dd.hip", "k_gram.hip", "k_rot.hip",
           "k_isvd.hip", "k_ttm.hip", "k_gramc.hip", "k_dense.hip", "k_eig.hip", "engine.hip", "tucker_ops.hip"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _hipcc():
    cand = os.path.join(ROCM, "bin", "hipcc")
    return cand if os.path.exists(cand) else (shutil.which("hipcc") or "hipcc")


def compile_flags():
    return [
        "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        "-Wno-unused-result",
    ]


# Per-source code generation options. The rotations and the fibre kernels keep
# their MFMA accumulators in VGPRs: with the default AGPR form the compiler
# copies the loop-carried accumulators between the two register files on every
# K block. (The Gram kernels keep the default: this compiler crashes on
# k_gram.hip with the VGPR form.)
_VGPR_FORM = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
SOURCE_FLAGS = {src: _VGPR_FORM for src in
                ("k_rot.hip", "k_fiber_ff.hip", "k_fiber_fd.hip", "k_fiber_dd.hip", "k_ttm.hip")}


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *compile_flags(), *SOURCE_FLAGS.get(src, []), "-c",
           os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose=False):
    """Compile all sources and link libstucker.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
           f"-L{ROCM}/lib", "-lrocsolver", "-lrocblas", f"-Wl,-rpath,{ROCM}/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
