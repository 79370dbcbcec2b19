"""Build the HIP library ``libknnf.so`` for gfx950 (in-tree, next to this file).

Usage: ``python -m paper_2404_10631_amd.build`` or ``build()`` from Python.

Flags that matter for the results:
* ``-ffp-contract=off`` and ``-fno-fast-math``: every ``*``, ``+``, ``-`` in the
  kernels is one IEEE binary32 operation; the only fused operations are the
  explicit ``fmaf`` calls of the distance.
* ``-fhip-fp32-correctly-rounded-divide-sqrt``: the Eq. 2 division is
  correctly rounded.
* ``-fno-gpu-flush-denormals-to-zero``: binary32 subnormals are kept.
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32
  instructions are generated.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libknnf.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["knnf_kernels.hip", "knnf_spectral.hip", "knnf_pc1.hip", "knnf_svm.hip", "knnf_api.cpp",
           "knnf_server.cpp"]

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))
ARCH = os.environ.get("KNNF_OFFLOAD_ARCH", "gfx950")

COMMON_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-Wno-unused-value",
    "-I", os.path.join(ROOT, "include"),
]
DEVICE_FLAGS = [
    f"--offload-arch={ARCH}",
    "-mcode-object-version=5",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    """Compile every source into ``libknnf.so`` (sources in parallel); returns its path."""
    from concurrent.futures import ThreadPoolExecutor

    cmds, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, src + ".o")
        cmd = [HIPCC] + COMMON_FLAGS + (extra or [])
        if src.endswith(".hip"):
            cmd += ["-x", "hip"] + DEVICE_FLAGS
        cmd += ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        for r in list(ex.map(lambda c: subprocess.run(c, check=True), cmds)):
            pass
    tmp = LIB + ".tmp"
    # roctx: the serving stages' trace ranges
    cmd = ([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
           + ["-L", os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx"])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
