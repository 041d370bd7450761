"""Build ``libsf.so`` (HIP, gfx950) in-tree with hipcc.

Each source compiles to an object in ``_build/`` in parallel, then one link
step makes ``paper_2407_06107_amd/libsf.so``.  Floating-point contraction is
off (the binary32 decision contract writes its fused operations explicitly)
and packed FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsf.so")
# Benchmark-only kernels (the gather-only twin of the stochastic ray march,
# the vector-ALU issue-rate probe), in a library of their own that no product
# path loads.
BENCH_SOURCES = ["bench_gather_twin.hip", "bench_valu_rates.hip"]
BENCH_LIB = os.path.join(PKG, "libsf_bench.so")

# Per-source flags: the neural decoder's matrix-core accumulators live in
# ordinary VGPRs (gfx950 MFMA accepts them), so the bias / ReLU / packing
# code that follows each layer reads them without AGPR-to-VGPR copies.
EXTRA_FLAGS = {"neural.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}

SOURCES = ["abi.hip", "filter2d.hip", "aniso.hip", "dct.hip", "triplanar.hip", "volume.hip", "neural.hip",
           "train.hip", "reduce.hip"]
ARCH = "gfx950"

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every HIP source for gfx950 and link libsf.so.  Always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *CFLAGS, *EXTRA_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(jobs, len(SOURCES) + len(BENCH_SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES + BENCH_SOURCES))
    for lib, part in ((LIB, objs[:len(SOURCES)]), (BENCH_LIB, objs[len(SOURCES):])):
        tmp = lib + ".tmp"
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *part, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link of {os.path.basename(lib)} failed:\n{r.stderr}")
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
