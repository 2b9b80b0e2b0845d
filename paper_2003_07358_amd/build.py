"""Builds libfhs.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2003_07358_amd.build         # or: python paper_2003_07358_amd/build.py

Every call recompiles.  Objects go to paper_2003_07358_amd/_build/ (ignored by
git); the library is paper_2003_07358_amd/libfhs.so.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfhs.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-I", BUILD]
# device code: gfx950 only; packed-FP32 instruction selection disabled
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".cpp", ".hip")) and f != "filtergen.cpp")


def gen_filters():
    """Compiles and runs filtergen (the library's own filter derivation) to
    write the compile-time tap header for the kernels."""
    exe = os.path.join(BUILD, "filtergen")
    cmd = ["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "filtergen.cpp"), os.path.join(CSRC, "hostmath.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"filtergen build failed:\n{r.stderr}")
    hdr = os.path.join(BUILD, "fhs_filters.h")
    r = subprocess.run([exe, hdr], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"filtergen failed:\n{r.stderr}")
    return hdr


def _compile(src, build_dir=BUILD, defines=()):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    flags = [*COMMON, *(f"-D{d}" for d in defines)]
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip", *DEVICE, *flags, "-c", src, "-o", obj]
    else:
        cmd = [HIPCC, *flags, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False, lib=LIB, defines=()):
    """Compiles every source and links `lib`.  `defines` (NAME=VALUE strings)
    override the launch-shape constants of the sources, for tuning builds."""
    os.makedirs(BUILD, exist_ok=True)
    gen_filters()
    bdir = BUILD if not defines else os.path.join(BUILD, "v_" + "_".join(defines).replace("=", ""))
    os.makedirs(bdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda src: _compile(src, bdir, defines), sources()))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                sys.stderr.write(err)
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
