"""Compile the native library ``libvecchia.so`` in-tree.

HIP sources (``csrc/*.hip``) are compiled for gfx950 only; the host graph
builder and the C-ABI glue (``csrc/*.cpp``) with g++ and no floating-point
contraction, so that the neighbour search rounds exactly as specified.  The
objects are linked by hipcc into one shared library next to this file.

Usage: ``python -m paper_2606_11402_amd.build`` (or ``build()`` from Python).
"""
import concurrent.futures
import glob
import os
import shlex
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libvecchia.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX_HOST", "g++")

HIP_FLAGS = [
    "-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
    "-I" + INCLUDE, "-I" + CSRC,
]
CXX_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-pthread", "-Wall",
             "-I" + INCLUDE, "-I" + CSRC]


def _run(cmd):
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if proc.returncode != 0:
        raise RuntimeError("build step failed:\n  %s\n%s" % (" ".join(shlex.quote(c) for c in cmd), proc.stdout))
    return proc.stdout


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, "-c", src, "-o", obj] + HIP_FLAGS
    else:
        cmd = [CXX, "-c", src, "-o", obj] + CXX_FLAGS
    _run(cmd)
    return obj


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _up_to_date(src):
    """An object is current when it is newer than its source and than every
    header it may include (all of csrc/*.h and include/*.h)."""
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return False
    deps = [src] + glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(INCLUDE, "*.h"))
    return os.path.getmtime(obj) > max(os.path.getmtime(d) for d in deps)


def build(jobs=None, verbose=False, incremental=False):
    """Compile every source and link ``libvecchia.so``.  By default every
    source is recompiled; incremental=True recompiles only the objects older
    than their source or a header."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(16, os.cpu_count() or 4)
    todo = [s for s in srcs if not (incremental and _up_to_date(s))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
         + ["-pthread", "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, "from", len(srcs), "sources")
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv[1:])
    sys.exit(0)
