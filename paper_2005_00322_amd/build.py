"""Build libpstd.so in-tree for gfx950 with hipcc (cross-compiles without a GPU).

Usage: ``python -m paper_2005_00322_amd.build`` (or ``build()`` from Python).  Always recompiles.
``python -m paper_2005_00322_amd.build --sanitize`` builds ``_build/sanitize/libpstd.so`` with the host
code under AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged), for running the
host-only entry points and argument checks under the sanitizers: load it with ``PSTD_LIBRARY`` set to its
path and the clang ASan runtime preloaded (``sanitizer_runtime()``).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libpstd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH, "-I" + os.path.join(ROOT, "include"),
          "-Wall", "-Wno-unused-result", "-Wno-unused-function", "-Wno-unused-variable"]
# hipcc -O3 forms packed FP32 instructions on its own; keep them off for all device code.
DEVICE_ONLY = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# host-side sanitizers only: each -fsanitize= applies to the host pass
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
            "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _compile(src: str, out_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + list(extra) + ["-c", src, "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
        cmd += DEVICE_ONLY
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out_dir = os.path.join(BUILD, "sanitize") if sanitize else BUILD
    lib = os.path.join(out_dir, "libpstd.so") if sanitize else LIB
    extra = SANITIZE if sanitize else []
    os.makedirs(out_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    workers = max(1, min(len(srcs), os.cpu_count() or 4, 8))
    with cf.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(lambda src: _compile(src, out_dir, extra), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + extra + ["-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, lib)
    if verbose:
        print("built", lib, file=sys.stderr)
    return lib


def sanitizer_runtime() -> str:
    """Path of the clang AddressSanitizer runtime hipcc links against (to preload into Python)."""
    r = subprocess.run([os.path.join(os.path.dirname(HIPCC), "..", "lib", "llvm", "bin", "clang"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
