"""Build libqst.so (gfx950) in-tree with hipcc.

    python -m paper_2207_05341_amd.build        # or __graft_entry__.build()

Every source is compiled to an object under paper_2207_05341_amd/_build/
(in parallel), then linked into paper_2207_05341_amd/libqst.so.  The HIP
code is compiled with packed-FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libqst.so")

SOURCES = ["qst_plan.cpp", "k_reduce.hip", "k_povm.hip", "k_povm_fast.hip", "k_gemm.hip", "qst_profile.hip", "k_batch.hip", "k_premap.hip", "k_fidelity.hip", "k_fnn.hip", "k_absmap.hip", "k_eigh.hip", "k_povm_general.hip", "k_xgemm.hip", "qst_api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found (ROCm toolchain required to build libqst)")
    return path


def common_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-Wall",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-I", CSRC,
    ]


# Per-source flags.  k_xgemm.hip: MFMA accumulators in VGPRs (the LLVM
# AMDGPU option selecting the VGPR form of the MFMA instructions).  With the
# default AGPR form the register allocator spills the split-bf16 products'
# FP32 chain totals to scratch memory; the reloads at every chain close are
# vector-memory loads queued behind the in-flight global-to-LDS copies of
# the operand ring, so each close waited for the whole ring.  In the VGPR
# form the totals spill to AGPRs and the MFMA loops are unchanged.
SOURCE_FLAGS = {"k_xgemm.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc(), *common_flags(), *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
