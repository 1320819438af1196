"""Build the HIP library libpm.so for gfx950 in-tree (hipcc, no JIT cache).

Every call recompiles: this is the "does it build" check as well as the way
the library is produced.  Objects are compiled in parallel and linked into
paper_2010_11847_amd/libpm.so next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpm.so")
ARCH = os.environ.get("PM_OFFLOAD_ARCH", "gfx950")

SOURCES = ["fft.hip", "particles.hip", "adjoint.hip", "recon.hip", "pyramid.hip", "api.cpp", "cosmo.cpp",
           "static_scratch.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# roctx ranges around the phases of a run (rocprofv3 --marker-trace)
LINK_LIBS = ["-lrocprofiler-sdk-roctx"]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _compile(src: str, build_dir: str) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        # the compiler's per-kernel resource report (registers, LDS, scratch)
        # is kept beside the object; a test rejects kernels that use scratch
        cmd = [HIPCC, *COMMON, *DEVICE, "-Rpass-analysis=kernel-resource-usage", "-c", path, "-o", obj]
    else:
        # host code; hipcc still runs a device pass over .cpp files, so name
        # the one target instead of its default architecture
        cmd = [HIPCC, *COMMON, f"--offload-arch={ARCH}", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if src.endswith(".hip"):
        with open(os.path.splitext(obj)[0] + ".usage.txt", "w") as fh:
            fh.write(r.stderr)
    return obj


def build(verbose: bool = False) -> str:
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, *LINK_LIBS, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


# Host code (api.cpp, cosmo.cpp and the host side of the .hip files) with
# AddressSanitizer and UndefinedBehaviorSanitizer; device code unchanged.
# The library is loaded with the sanitizer runtime preloaded (CPU tests of
# the host logic: validation, workspace layout, the host tables).
SANITIZE = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
HOST_SANITIZED_LIB = os.path.join(HERE, "_build", "host_sanitized", "libpm_hostsan.so")


def sanitizer_runtime() -> str:
    """Path of the clang AddressSanitizer runtime that hipcc's host compiler uses."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


def build_host_sanitized(verbose: bool = False) -> str:
    build_dir = os.path.dirname(HOST_SANITIZED_LIB)
    os.makedirs(build_dir, exist_ok=True)

    def comp(src):
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        dev = DEVICE if src.endswith(".hip") else [f"--offload-arch={ARCH}"]
        cmd = [HIPCC, *COMMON, *dev, *SANITIZE, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        objs = list(ex.map(comp, srcs))
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *SANITIZE, *objs, *LINK_LIBS, "-o", HOST_SANITIZED_LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(f"built {HOST_SANITIZED_LIB}", file=sys.stderr)
    return HOST_SANITIZED_LIB


if __name__ == "__main__":
    build(verbose=True)
