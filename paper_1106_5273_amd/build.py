"""Compile the HIP library libvfmm.so in-tree for gfx950 with hipcc.

Every HIP translation unit is built with packed-FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops).  Objects go to _build/
next to this file; the shared library is written next to this file.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libvfmm.so")
MB_OUT = os.path.join(HERE, "libvfmm_mb.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "tree.hip", "traverse.hip", "far.hip", "m2lb.hip", "p2p.hip", "autotune.hip",
           "direct_static.hip", "rbf.hip", "spectrum.hip", "lattice_host.cpp"]
ARCH = os.environ.get("VFMM_ARCH", "gfx950")


def hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


def compile_one(src, verbose):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc()] + flags() + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: compile_one(s, verbose), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    # VALU-rate microbenchmarks: a separate small library, not part of the C ABI
    mb = compile_one("microbench.hip", verbose)
    tmp = MB_OUT + ".tmp"
    subprocess.check_call([hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp, mb])
    os.replace(tmp, MB_OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(OUT)
