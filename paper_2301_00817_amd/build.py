"""Build liblesjet.so in-tree with hipcc for gfx950.

    python -m paper_2301_00817_amd.build          # compile everything

Objects go to paper_2301_00817_amd/_build/, the library to
paper_2301_00817_amd/_lib/liblesjet.so.  Compilation is parallel over the
source files and always redone (the build is the 'does it compile' check).
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "liblesjet.so")
ARCH = os.environ.get("LESJET_ARCH", "gfx950")

SOURCES = ["api.cpp", "geometry.hip", "ghost.hip", "residual_ref.hip", "residual_fused.hip",
           "rk.hip", "diag.hip", "adjoint.hip", "dynamic.hip"]

CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# Per-source flags.  The stage kernel (bound by latency in FP64) is scheduled
# for instruction-level parallelism: 1 % less time per FP64 launch on MI355X,
# FP32 and the other kernels unchanged.
SOURCE_FLAGS = {"residual_fused.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src, build_dir=BUILD, defines=()):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *CFLAGS, *SOURCE_FLAGS.get(src, []), *[f"-D{d}" for d in defines], "-c",
           os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-x")
        cmd.insert(2, "hip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
    return obj, r.stderr


CHECKS_SRC = os.path.join(ROOT, "tests", "host_checks.hip")
CHECKS_LIB = os.path.join(LIBDIR, "liblesjet_checks.so")


def build_checks():
    """Host-compiled check library of the device functions (test helper)."""
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = CHECKS_LIB + ".tmp"
    cmd = [_hipcc(), *CFLAGS, "-shared", "-x", "hip", CHECKS_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on host_checks.hip:\n{r.stderr[-6000:]}")
    os.replace(tmp, CHECKS_LIB)
    return CHECKS_LIB


def build(verbose=False, lib=LIB, defines=()):
    """Compile all sources and link `lib`; `defines` are extra -D macros
    (variants for measurements, built to another path)."""
    build_dir = BUILD if lib == LIB else os.path.join(os.path.dirname(os.path.abspath(lib)), "_obj")
    os.makedirs(build_dir, exist_ok=True)
    os.makedirs(os.path.dirname(os.path.abspath(lib)), exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(lambda src: _compile(src, build_dir, defines), SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", "-Wl,--no-undefined", "-o", tmp,
           *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, lib)
    if lib == LIB and os.path.exists(CHECKS_SRC):
        build_checks()
    return lib


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=LIB)
    ap.add_argument("-D", dest="defines", action="append", default=[])
    a = ap.parse_args()
    print(build(verbose=True, lib=a.out, defines=a.defines))
