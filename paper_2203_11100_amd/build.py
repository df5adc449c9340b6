"""Builds libswdb.so (HIP kernels for gfx950 + host runtime) in place.

    python -m paper_2203_11100_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libswdb.so")
SOURCES = ["layout.cpp", "runtime.hip", "k_inter.hip", "k_batch.hip", "k_intra.hip", "k_misc.hip", "k_hits.hip", "k_modes.hip",
           "cpu_scorer.cpp", "trace_walk.cpp"]
HOST_SOURCES = ("cpu_scorer.cpp", "trace_walk.cpp")
ARCH = os.environ.get("SWDB_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def build(verbose: bool = True, jobs: int = 8) -> str:
    objs = []
    procs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src.replace(".", "_") + ".o")
        if src in HOST_SOURCES:      # host-only C++ (no device code)
            cmd = [hipcc(), "-x", "c++", "-O3", "-std=c++17", "-fPIC", "-Wall",
                   "-c", os.path.join(CSRC, src), "-o", obj]
        else:
            cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-Wall", "-Wno-unused-function", "-x", "hip",
                   "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    failed = False
    for p, src in procs:
        _, err = p.communicate()
        lines = [ln for ln in err.splitlines() if "packed-fp32-ops" not in ln]
        if lines:
            print("\n".join(lines), file=sys.stderr)
        if p.returncode != 0:
            failed = True
            print("compile failed: %s" % src, file=sys.stderr)
    if failed:
        raise RuntimeError("libswdb build failed")
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o",
           LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build()
