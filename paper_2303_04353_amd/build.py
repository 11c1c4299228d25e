"""Build the HIP library ``libddgemm.so`` (gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libddgemm.so")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
ARCH = os.environ.get("DDGEMM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    # IEEE FP64 semantics the split and the FP64x2 arithmetic rely on: no
    # contraction of a*b+c, no fast-math reassociation.
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "not a recognized feature for this target"
    msg = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if noise not in l and l.strip())
    return res.returncode, msg


def build(verbose: bool = False) -> str:
    """Compile every source to an object in ``_build/`` (in parallel), then
    link ``libddgemm.so``.  Always compiles: the result is what the sources
    say now."""
    os.makedirs(BUILD, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    jobs = []
    for src in sources():
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        jobs.append((["hipcc", *compile_flags, "-c", src, "-o", obj], obj))
    workers = min(len(jobs), max(1, min(8, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda j: _run(j[0]), jobs))
    for (cmd, _), (rc, msg) in zip(jobs, results):
        if verbose:
            print(" ".join(cmd), flush=True)
            if msg:
                print(msg)
        if rc != 0:
            raise RuntimeError("hipcc failed:\n" + msg)
    tmp = LIB + ".tmp%d" % os.getpid()
    # rocBLAS: the plain FP64 GEMMs of the unfused comparator form
    cmd = ["hipcc", *HIPCC_FLAGS, *[o for _, o in jobs], "-o", tmp, "-lrocblas"]
    if verbose:
        print(" ".join(cmd), flush=True)
    rc, msg = _run(cmd)
    if rc != 0:
        raise RuntimeError("link failed:\n" + msg)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
