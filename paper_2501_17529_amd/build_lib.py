"""Compile the HIP sources into the in-tree shared library libdcflow.so (gfx950).

Usage: python -m paper_2501_17529_amd.build_lib   (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdcflow.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["abi.hip", "build.hip", "factors.hip", "inject.hip", "score.hip", "percase.hip",
           "mlp.hip", "mlp_abi.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 VALU forms are kept off: every kernel is written for the
         # unpacked FP32 FMA / max instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA sources and results in ordinary VGPRs (no AGPR copies): the scan
         # consumes each L~ block with VALU instructions right after it is built
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-Wno-unused-result"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
