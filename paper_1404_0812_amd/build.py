"""Build librbffd.so for gfx950 with hipcc (in-tree, next to this file).

    python -m paper_1404_0812_amd.build [--verbose] [--incremental]
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "librbffd.so")
ARCH = os.environ.get("RBFFD_ARCH", "gfx950")

# (source, object name, defines); the weights kernels are built once per
# (radial kernel, tiling) so that the six large variants compile in parallel.
# Longest first.
SOURCES = [("weights_kernels.hip", f"weights_k{k}_nb{nb}", [f"-DRBW_K={k}", f"-DRBW_NB={nb}"])
           for nb in (2, 1) for k in (0, 1, 2)]
SOURCES += [("weights_dd.hip", "weights_dd", []), ("mlp.hip", "mlp", []), ("step.hip", "step", []), ("grid_knn.hip", "grid_knn", []),
            ("context.cpp", "context", []), ("batched.cpp", "batched", []), ("weights.cpp", "weights", [])]

# Packed FP32 instructions are disabled for all device code: the compiler
# otherwise forms v_pk_* FP32 operations from scalar float code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# The weights kernels keep the local matrix in registers and index it only
# with loop counters of fully unrolled loops; the default size limit of a
# full unroll would leave the largest loops rolled and the matrix in scratch.
UNROLL_FLAGS = ["-mllvm", "-pragma-unroll-threshold=200000"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def _newest_dependency(src: str) -> float:
    deps = [os.path.join(CSRC, src), os.path.join(INCLUDE, "rbffd.h"), os.path.abspath(__file__)]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    return max(os.path.getmtime(d) for d in deps)


def _compile(entry, verbose: bool, incremental: bool = False) -> str:
    src, name, defines = entry
    obj = os.path.join(BUILD, name + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _newest_dependency(src):
        return obj
    cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC]
    cmd += DEVICE_FLAGS + defines
    if src.endswith(".hip"):
        cmd += ["-munsafe-fp-atomics"] + UNROLL_FLAGS
        if os.environ.get("RBFFD_RESOURCE_USAGE"):
            cmd += ["-Rpass-analysis=kernel-resource-usage"]
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only those older than their
    source or any header) and link librbffd.so."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv, incremental="--incremental" in sys.argv))
