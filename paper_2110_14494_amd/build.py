"""Builds the HIP library libpcmcc.so for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpcmcc.so")
SOURCES = ["pcmcc_kernels.hip", "pcmcc_deposit.hip", "pcmcc_weights.hip", "pcmcc_swarm.hip", "pcmcc_mlp.hip",
           "pcmcc_field.hip", "pcmcc_fluid.hip", "pcmcc_photo.hip", "pcmcc_runtime.hip", "pcmcc_api.hip", "pcmcc_noalloc.hip",
           "pcmcc_api_swarm.hip", "pcmcc_api_mlp.hip", "pcmcc_api_field.hip", "pcmcc_api_fluid.hip"]
ARCH = os.environ.get("PCMCC_OFFLOAD_ARCH", "gfx950")
CONTRACT_OFF = ("pcmcc_kernels.hip", "pcmcc_swarm.hip")
# matrix-instruction accumulators in ordinary vector registers: the
# surrogate's inference then needs no accumulator-register reads and fits
# five waves per SIMD (86 registers instead of 116)
MFMA_VGPR = ("pcmcc_mlp.hip",)


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> str:
    """Compiles every HIP source and links libpcmcc.so (always rebuilds)."""
    objs = []
    flags = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        # the electron mover's arithmetic is exactly what its source writes
        # (explicit fused multiply-adds only): implicit contraction may fuse
        # a sum of products either way, so an unrelated code change could
        # move results by an ulp
        extra = ["-ffp-contract=off"] if src in CONTRACT_OFF else []
        if src in MFMA_VGPR:
            extra += ["-mllvm", "-amdgpu-mfma-vgpr-form"]
        cmd = [hipcc()] + flags + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
