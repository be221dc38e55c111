"""Build librgdbek.so (HIP kernels + C++ runtime) for gfx950 with hipcc.

Usage: python -m paper_2509_19267_amd.build   (or build() from Python).
Objects go to paper_2509_19267_amd/_build/, the library to
paper_2509_19267_amd/_lib/librgdbek.so.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "_lib")
LIBNAME = "librgdbek.so"
ARCH = "gfx950"

SOURCES = ["select.hip", "spmv.hip", "proj.hip", "utils.hip", "batch.hip",
           "rep.hip", "runtime.hip"]
# Bit-exact selection needs unfused, correctly rounded FP64 operations.
EXTRA = {"select.hip": ["-ffp-contract=off"]}


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc",
              shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build)")


def common_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(HERE, "..", "include"), "-I" + CSRC]


def _compile(src):
    out = os.path.join(OBJ, src.replace(".hip", ".o"))
    cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", out] + \
        common_flags() + EXTRA.get(src, [])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{r.stderr[-6000:]}")
    return out


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(LIB, exist_ok=True)
    workers = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = os.path.join(LIB, LIBNAME + ".tmp")
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + \
        ["--offload-arch=" + ARCH, "-fPIC"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, os.path.join(LIB, LIBNAME))
    if verbose:
        print("built", os.path.join(LIB, LIBNAME))
    return os.path.join(LIB, LIBNAME)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
