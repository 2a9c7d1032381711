"""Builds libgsim.so (HIP kernels + host runtime + C-ABI) for gfx950 with hipcc.

Usage: ``python -m paper_2104_02646_amd.build`` (the repository's
``__graft_entry__.build()`` calls :func:`build`).  The library is written
in-tree next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libgsim.so")
SOURCES = ["gsim_kernels.hip", "gsim_control.hip", "gsim_rigid.hip", "gsim_raster.hip", "gsim_api.cpp", "gsim_engine.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU ops.
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", INCLUDE]


# Host-only sanitizers for the host runtime (planner, call drivers, engine): each flag is
# given to the host pass alone; device code is compiled as in the plain build.
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
HOST_SOURCES = ["gsim_api.cpp", "gsim_engine.cpp"]
CLANGXX = os.environ.get("GSIM_CLANGXX", "/opt/rocm/llvm/bin/clang++")


def asan_runtime() -> str:
    """The clang ASan runtime a non-instrumented host process (Python) preloads to load
    the sanitizer build."""
    import glob
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise FileNotFoundError("clang ASan runtime not found under /opt/rocm/llvm")
    return found[-1]


def build_sanitized(out_dir: str, verbose: bool = False) -> str:
    """Builds out_dir/libgsim.so with the host runtime (gsim_api.cpp, gsim_engine.cpp)
    under AddressSanitizer and UndefinedBehaviorSanitizer (aborting on the first report),
    linked with the kernel objects of the plain build.  Load it from Python with
    GSIM_LIB=<path> and the runtime from :func:`asan_runtime` in LD_PRELOAD."""
    os.makedirs(out_dir, exist_ok=True)
    kobjs = [os.path.join(CSRC, s.rsplit(".", 1)[0] + ".o") for s in SOURCES if s not in HOST_SOURCES]
    if not all(os.path.exists(o) for o in kobjs):
        build(verbose)
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, src.rsplit(".", 1)[0] + ".san.o")
        cmd = [HIPCC, *[f.replace("-O3", "-O1") for f in FLAGS], *SAN_HOST, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    lib = os.path.join(out_dir, "libgsim.so")
    link = [CLANGXX, "-shared", "-fPIC", "-shared-libasan"]
    link += ["-fsanitize=" + s for s in ("address", "undefined")]
    link += [*objs, *kobjs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", lib]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    return lib


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.rsplit(".", 1)[0] + ".o")
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-z,defs", *objs, "-o", tmp]  # no undefined symbols
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        out = [a for a in sys.argv[1:] if not a.startswith("-")]
        print(build_sanitized(out[0] if out else os.path.join(HERE, "_build", "san"), verbose="-v" in sys.argv))
    else:
        build(verbose="-v" in sys.argv)
        print(LIB)
