"""Build libmhdlbm.so (gfx950 HIP kernels + host runtime) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmhdlbm.so")
SOURCES = ["mhd_sweep.hip", "mhd_kernels.hip", "mhd_noalloc.hip", "mhd_runtime.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    """Compile the sources to objects in parallel, then link libmhdlbm.so (always rebuilds)."""
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    objs = [os.path.join(CSRC, s + ".o") for s in SOURCES]
    noise = "packed-fp32-ops"

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
        if verbose and err.strip():
            print(err)

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(run, [[hipcc, *compile_flags, "-c", os.path.join(CSRC, s), "-o", o]
                          for s, o in zip(SOURCES, objs)]))
    run([hipcc, *HIPCC_FLAGS, *objs, "-o", LIB + ".tmp"])
    for o in objs:
        os.remove(o)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
