"""Build libprune_hip.so (HIP for gfx950) in-tree with hipcc.

Every translation unit under csrc/ is compiled as HIP for gfx950 with
packed-FP32 instructions disabled (-target-feature -packed-fp32-ops) and
matrix-core accumulators selected in VGPR form, then linked into
paper_1802_06625_amd/libprune_hip.so.  A second library,
libprune_hip_debug.so, is built from the same sources with PRUNE_DEBUG
defined: its bookkeeping kernels check the FIFO invariants after every
counter update.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libprune_hip.so")
OUT_DEBUG = os.path.join(HERE, "libprune_hip_debug.so")
BUILD_DIR = os.path.join(HERE, "_build")

ARCH = os.environ.get("PRUNE_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core accumulators in ordinary VGPRs (gfx950 MFMA takes them as
    # C/D operands): no accumulator copies between AGPRs and VGPRs in loops
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src: str, verbose: bool, debug: bool) -> str:
    out_dir = os.path.join(BUILD_DIR, "debug") if debug else BUILD_DIR
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [hipcc(), "-x", "hip", "-c", src, "-o", obj] + FLAGS + (["-DPRUNE_DEBUG"] if debug else [])
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stdout}\n{res.stderr}")
    warn = "\n".join(l for l in res.stderr.splitlines()
                     if "packed-fp32-ops" not in l and "not a recognized feature" not in l
                     and l.strip())
    if warn and verbose:
        print(warn, file=sys.stderr)
    return obj


def _link(objs, out: str) -> None:
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False, debug: bool = True) -> str:
    """Compile and link libprune_hip.so and, with debug, libprune_hip_debug.so."""
    os.makedirs(os.path.join(BUILD_DIR, "debug"), exist_ok=True)
    srcs = sources()
    kinds = [False, True] if debug else [False]
    jobs = [(s, d) for d in kinds for s in srcs]
    with cf.ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:
        objs = list(ex.map(lambda j: _compile(j[0], verbose, j[1]), jobs))
    _link(objs[:len(srcs)], OUT)
    if debug:
        _link(objs[len(srcs):], OUT_DEBUG)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
