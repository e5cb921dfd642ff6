"""Build libgmrf.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1606_00980_amd.build              # libgmrf.so
    python -m paper_1606_00980_amd.build --sanitize   # also libgmrf_san.so

Every call recompiles all sources; object files go to ``_build/`` beside this
file and the shared library to ``libgmrf.so``.

``--sanitize`` (or ``build_sanitized()``) builds ``libgmrf_san.so``: the host
runtime (the ``.cpp`` sources: argument validation, planning, the serving
loop) compiled with AddressSanitizer and UndefinedBehaviorSanitizer on the
host side only, linked with the kernel objects of the plain build.  It is for
host-side checks on the CPU: load it with ``GMRF_LIB=<path>`` and the
sanitizer runtime preloaded (``sanitizer_runtime()``).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libgmrf.so")
OUT_SAN = os.path.join(HERE, "libgmrf_san.so")
BUILD = os.path.join(HERE, "_build")
BUILD_SAN = os.path.join(BUILD, "san")

SOURCES = ["k_pcg_f32.hip", "k_pcg_f64.hip", "k_ops.hip", "k_rng.hip", "k_data.hip", "k_rbic_f32.hip",
           "k_rbic_f64.hip", "api.cpp", "server.cpp", "tune.cpp", "data.cpp", "rbic.cpp"]

ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]


# Host-side sanitizers only (device code is never instrumented).
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-g"]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP toolchain is required to build libgmrf.so")
    return path


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD_SAN if sanitize else BUILD, os.path.splitext(src)[0] + ".o")
    extra = SAN_FLAGS if sanitize else []
    cmd = [hipcc(), *COMMON, *DEVICE_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc(), "-x", "hip", *COMMON, *DEVICE_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    msg = "\n".join(line for line in (res.stdout + res.stderr).splitlines() if noise not in line)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{msg}")
    if msg.strip():
        print(msg, file=sys.stderr)
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}{res.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


def build_sanitized(verbose: bool = True, out: str = OUT_SAN) -> str:
    """libgmrf_san.so (at `out`) from the host sources compiled with
    sanitizers and the kernel objects of build() (built first if they are
    missing)."""
    kernels = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(k) for k in kernels):
        build(verbose=verbose)
    os.makedirs(BUILD_SAN, exist_ok=True)
    hosts = [s for s in SOURCES if s.endswith(".cpp")]
    with ThreadPoolExecutor(max_workers=min(len(hosts), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, True), hosts))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *kernels, *objs, *SAN_FLAGS, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}{res.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


def sanitizer_runtime() -> str:
    """The compiler's AddressSanitizer runtime (it carries the
    UndefinedBehaviorSanitizer handlers too), to preload into a process that
    loads libgmrf_san.so."""
    res = subprocess.run([os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "lib", "llvm", "bin",
                                       "clang"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("the AddressSanitizer runtime of the HIP compiler was not found")
    return path


if __name__ == "__main__":
    build()
    if "--sanitize" in sys.argv[1:]:
        build_sanitized()
