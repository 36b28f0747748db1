"""Compile libgenie.so for gfx950 with hipcc (in-tree, next to this file).

Each source compiles to its own object (in parallel), then one link."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/api.cpp", "csrc/search.hip", "csrc/lsh.hip", "csrc/gate.hip", "csrc/timing.cpp",
           "csrc/parts.cpp", "csrc/sequence.hip", "csrc/probe.hip"]
LIB = os.path.join(HERE, "libgenie.so")
OBJ_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
NOISE = "is not a recognized feature for this target"


def _run(cmd):
    proc = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (proc.stderr or "").splitlines() if NOISE not in l)
    return proc.returncode, err


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    jobs = []
    for s in SOURCES:
        obj = os.path.join(OBJ_DIR, os.path.basename(s) + ".o")
        jobs.append(([HIPCC] + FLAGS + inc + ["-c", os.path.join(HERE, s), "-o", obj], obj))
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    with cf.ThreadPoolExecutor(workers) as pool:
        results = list(pool.map(lambda j: _run(j[0]), jobs))
    for (cmd, _), (rc, err) in zip(jobs, results):
        if verbose:
            print(" ".join(cmd), flush=True)
        if rc != 0:
            raise RuntimeError(f"hipcc failed ({rc}):\n{err}")
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for _, o in jobs] + ["-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    rc, err = _run(link)
    if rc != 0:
        raise RuntimeError(f"hipcc link failed ({rc}):\n{err}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
