"""Builds libgodiet.so (the HIP library for gfx950) in-tree with hipcc: every source is
compiled to an object in parallel, then the objects are linked."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgodiet.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["gd_api.hip", "gd_scan.hip", "gd_sketch.hip", "gd_sort.hip", "gd_seed.hip",
           "gd_trace.hip", "gd_rmi.hip", "gd_contain.hip", "gd_vote.hip", "gd_table.hip",
           "gd_fig4.hip"]

OBJ_DIR = os.path.join(HERE, "_build")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # no packed-FP32 instructions anywhere in the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _run(cmd, verbose, what):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + what)


def build(verbose=False):
    """Compile every source and link libgodiet.so; always rebuilds."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = []
    jobs = []
    for src in SOURCES:
        obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        jobs.append(([hipcc()] + FLAGS + ["-I", INCLUDE, "-I", CSRC, "-c",
                      os.path.join(CSRC, src), "-o", obj], src))
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda j: _run(j[0], verbose, j[1]), jobs))
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose,
         "libgodiet.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
