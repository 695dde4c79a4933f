"""Builds libmlp.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1908_07847_amd.build

Every source under csrc/ is compiled to an object in _build/ (in parallel),
then linked into paper_1908_07847_amd/libmlp.so.  Packed FP32 VALU
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmlp.so")
ARCH = os.environ.get("MLP_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC, "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, "-c", src, "-o", obj] + CFLAGS
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip", "-c", src, "-o", obj] + CFLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    noise = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
    if noise:
        sys.stderr.write("\n".join(noise) + "\n")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources for {ARCH}")
    return LIB


ASAN_LIB = os.path.join(BUILD, "libmlp_asan.so")


def asan_runtime() -> str:
    """The compiler's host AddressSanitizer runtime (to preload into a Python
    process that loads the sanitized library)."""
    r = subprocess.run([HIPCC.replace("hipcc", "amdclang++") if HIPCC.endswith("hipcc") else HIPCC,
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return path
    import glob
    found = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise RuntimeError("no host AddressSanitizer runtime found")
    return found[-1]


def build_asan() -> str:
    """A copy of the library whose host code (the C ABI layer, mlp_api.cpp)
    is built with AddressSanitizer; the device code and the kernels' host
    stubs are the regular objects.  For the ABI tests on the host only: it is
    loaded through MLP_LIBRARY with the runtime preloaded, never shipped."""
    if not all(os.path.exists(os.path.join(BUILD, os.path.basename(f) + ".o")) for f in sources()):
        build(verbose=False)
    api = os.path.join(CSRC, "mlp_api.cpp")
    obj = os.path.join(BUILD, "mlp_api_asan.o")
    flags = [f if f != "-O3" else "-O1" for f in CFLAGS] + ["-g", "-Xarch_host", "-fsanitize=address",
                                                            "-Xarch_host", "-fno-omit-frame-pointer"]
    r = subprocess.run([HIPCC, "-x", "hip", "-c", api, "-o", obj] + flags, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {api}:\n{r.stderr}")
    others = [os.path.join(BUILD, os.path.basename(f) + ".o") for f in sources() if not f.endswith("mlp_api.cpp")]
    tmp = ASAN_LIB + ".tmp%d" % os.getpid()
    r = subprocess.run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
                        "-Xarch_host", "-shared-libasan", "-o", tmp, obj] + others, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


if __name__ == "__main__":
    build()
