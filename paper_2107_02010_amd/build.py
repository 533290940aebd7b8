"""Builds libskh.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc.

    python -m paper_2107_02010_amd.build

The library lands next to this file; the Python binding loads it from there.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libskh.so")
# issue-rate probe behind the ALU ceilings of the bench's 3-D and p-cost lines
PROBE_SRC = os.path.join(CSRC, "valu_probe.hip")
PROBE = os.path.join(HERE, "valu_probe")

SOURCES = ["softmin.hip", "softmin_bf16.hip", "softmin_pcost.hip", "plan.hip", "kmeans.hip", "multiscale.hip",
           "aux_kernels.hip", "warmstart.hip", "api.cpp", "ws_api.cpp"]
ARCH = os.environ.get("SKH_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are kept out of the generated code; hipcc's host
# pass warns that it does not know the feature, which is harmless.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-mllvm", "-amdgpu-mfma-vgpr-form",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libskh)")


def _compile(cc: str, src: str, obj: str, verbose: bool) -> None:
    cmd = [cc, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compiles every source (in parallel) and links libskh.so in place."""
    from concurrent.futures import ThreadPoolExecutor
    cc = hipcc()
    tmpdir = tempfile.mkdtemp(prefix="skh_build_")
    try:
        objs = [os.path.join(tmpdir, src + ".o") for src in SOURCES]
        workers = jobs or min(len(SOURCES), os.cpu_count() or 1, 8)
        with ThreadPoolExecutor(max_workers=workers) as ex:
            for f in [ex.submit(_compile, cc, src, obj, verbose) for src, obj in zip(SOURCES, objs)]:
                f.result()
        tmp_lib = LIB + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib, *objs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(tmp_lib, LIB)
        cmd = [cc, *HIP_FLAGS, "-x", "hip", PROBE_SRC, "-o", PROBE + ".tmp"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on valu_probe.hip:\n{r.stderr}")
        os.replace(PROBE + ".tmp", PROBE)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
