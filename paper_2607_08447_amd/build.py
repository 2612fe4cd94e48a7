"""Build the HIP library libhkp.so for gfx950 (in-tree).

    python -m paper_2607_08447_amd.build        (or python paper_2607_08447_amd/build.py)

Every source is compiled by hipcc for gfx950 only, with packed FP32
instructions disabled, and linked into paper_2607_08447_amd/libhkp.so.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhkp.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["stencil.hip", "stencil2.hip", "fields.hip", "blas.hip", "eig.hip", "sp.hip", "spinfree.hip",
           "gmatrix.hip",
           "solver.cpp",
           "sp_loop.cpp", "abi.cpp", "autotune.cpp"]

FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA accumulators in VGPRs: the AGPR form made the compiler copy every
         # loop-carried accumulator AGPR <-> VGPR around each MFMA
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I", os.path.join(ROOT, "include"), "-I", SRC, "-Wall", "-Wno-unused-function",
         "-Wno-unused-variable", "-Wno-unused-but-set-variable"]


def _compile(src):
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(SRC, src), "-o", out]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(SRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    return out, warn


# host sources whose argument validation the sanitizer build checks
ASAN_SOURCES = ["abi.cpp", "autotune.cpp", "solver.cpp", "sp_loop.cpp"]
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
ASAN_LIB = os.path.join(HERE, "libhkp_asan.so")


def _compile_asan(src):
    out = os.path.join(OBJ, "asan_" + os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ASAN_FLAGS + ["-x", "hip", "-c", os.path.join(SRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def build_asan():
    """libhkp_asan.so: the host sources above built with AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only), linked with the kernels' objects
    of the normal build (build() first).  Loaded by a CPU test in a process that
    preloads the sanitizer runtime."""
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(ASAN_SOURCES)) as ex:
        objs = list(ex.map(_compile_asan, ASAN_SOURCES))
    plain = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in SOURCES
             if s not in ASAN_SOURCES]
    tmp = ASAN_LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-fsanitize=address,undefined",
           "-shared-libsan", "-o", tmp] + objs + plain
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    if verbose:
        for _, w in results:
            if w:
                print(w, file=sys.stderr)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
