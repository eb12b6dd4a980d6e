"""Build libslista.so (the HIP library behind include/slista.h) for gfx950.

Run `python -m paper_1905_11071_amd.build` or call build(). Compiles every
source under csrc/ with hipcc, in-tree, and links them into
paper_1905_11071_amd/libslista.so.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libslista.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: no v_pk_{add,mul,fma}_f32 in device code (the host pass
# warns that it does not know the feature; that is expected).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                # the persistent kernels unroll their column passes fully so that the
                # master iterate stays in registers (the default limit leaves it in scratch)
                "-mllvm", "-pragma-unroll-threshold=1000000"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-fvisibility=hidden", "-Wall", "-Wno-unused-result",
          f"-I{os.path.join(ROOT, 'include')}"]

SOURCES = ["kernels_persist_bf16.hip", "kernels_persist_f32.hip", "kernels_gemm.hip", "kernels_misc.hip",
           "kernels_lista.hip", "kernels_lista_persist.hip", "kernels_persist.hip", "kernels_check.hip",
           "kernels_f64.hip", "api.cpp"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD_DIR, src + ".o")
    # api.cpp holds host code only; the same target keeps hipcc's device pass on gfx950
    cmd = [HIPCC] + COMMON + [f"--offload-arch={ARCH}"] + DEVICE_FLAGS
    cmd += ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile all sources and link libslista.so. Returns the library path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
