"""Build liblbfd_hip.so (the C-ABI library) for gfx950 with hipcc.

The FP64 kernels are compiled without floating-point contraction so that the
FP64 mode evaluates the same roundings as a plain CPU implementation would;
the FP32 kernels keep the default contraction (fused multiply-add).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblbfd_hip.so")
ARCH = "gfx950"

COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
UNITS = [
    # matrix-product accumulators in ordinary VGPRs (the surrogate kernels'
    # epilogues read them directly)
    ("lbfd_kernels_f32.hip", ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]),
    ("lbfd_kernels_f64.hip", ["-ffp-contract=off"]),
    ("lbfd_runtime.hip", []),
    ("lbfd_train.hip", []),
]


def _compile(unit):
    src, extra = unit
    obj = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
    cmd = ["hipcc"] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(UNITS)) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
