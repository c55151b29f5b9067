"""Build libepr.so (HIP, gfx950) in the package directory.

    python -m paper_2601_22793_amd.build [-v] [--host-asan]

Every translation unit under csrc/ is compiled with hipcc for gfx950 into _build/, in
parallel, then linked into paper_2601_22793_amd/libepr.so.  The build always recompiles.

--host-asan builds _build/asan/libepr_asan.so instead: the same sources with the host code
instrumented by AddressSanitizer (device code is built as usual), linked with clang++ against
the shared sanitizer runtime.  A process loads it with that runtime preloaded (ASAN_RUNTIME)
and EPR_LIBRARY naming it; the package never loads it by itself.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libepr.so")
# the library exports the C ABI (epr_*) only
EXPORTS = "-Wl,--version-script=" + os.path.join(CSRC, "libepr.map")

SOURCES = ["host_core.cpp", "api_ops.cpp", "api_solve.cpp", "api_batch.cpp", "api_tune.cpp", "k_transport.hip", "k_spectral.hip", "k_local.hip", "k_vjp.hip",
           "k_regime.hip", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code.
FLAGS = [
    "-x", "hip", "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


LLVM = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm")
# host-only instrumentation: every sanitizer flag applies to the host pass alone
ASAN_FLAGS = "-Xarch_host -fsanitize=address -Xarch_host -fno-omit-frame-pointer -Xarch_host -g".split()
ASAN_BUILD = os.path.join(BUILD, "asan")
ASAN_LIB = os.path.join(ASAN_BUILD, "libepr_asan.so")


def asan_runtime():
    """Path of the clang AddressSanitizer runtime the host-ASan build links against."""
    r = subprocess.run([os.path.join(LLVM, "bin", "clang++"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("clang's AddressSanitizer runtime was not found")
    return path


def _compile(src, verbose, out_dir=BUILD, extra=()):
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    noise = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if verbose and noise:
        print("\n".join(noise), flush=True)
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, EXPORTS, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def build_host_asan(verbose=False):
    """Build ASAN_LIB (host code under AddressSanitizer) and return its path."""
    os.makedirs(ASAN_BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, ASAN_BUILD, ASAN_FLAGS), SOURCES))
    rt = asan_runtime()
    tmp = ASAN_LIB + ".tmp"
    cmd = [os.path.join(LLVM, "bin", "clang++"), "-shared", "-fPIC", *objs, rt, EXPORTS,
           "-Wl,-rpath," + os.path.dirname(rt), "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


if __name__ == "__main__":
    if "--host-asan" in sys.argv:
        print(build_host_asan(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
