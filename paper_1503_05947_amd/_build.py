"""Compile the HIP sources of the library into ``librbd.so`` next to this file.

gfx950 only.  Packed FP32 instructions are disabled for every HIP translation
unit; the host pass warns that it does not know that target feature, which is
harmless.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librbd.so")
SOURCES = ["rbd_api.hip", "rbd_batched.hip", "rbd_backward.hip", "rbd_classify.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def build_library(verbose: bool = False) -> str:
    """Always recompiles; writes to a temporary name and renames atomically."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    if verbose:
        noise = [l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l]
        if noise:
            print("\n".join(noise))
    os.replace(tmp, LIB)
    return LIB


SANITIZED_LIB = os.path.join(HERE, "_build", "librbd_hostsan.so")
SANITIZER_FLAGS = [
    # host code only: each -fsanitize= goes to the host pass; device code is built as usual
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer",
    "-shared-libasan", "-g",
]


def asan_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (to be preloaded by an
    uninstrumented host program such as python)."""
    res = subprocess.run([hipcc(), "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
        import glob
        hits = glob.glob(os.path.join(rocm, "lib", "llvm", "lib", "clang", "*", "lib", "linux",
                                      "libclang_rt.asan-x86_64.so"))
        path = hits[0] if hits else ""
    if not path:
        raise RuntimeError("libclang_rt.asan-x86_64.so not found")
    return path


def build_host_sanitized() -> str:
    """The same library with its host code (argument checks, launch plans,
    workspace layout, batch plans) built under AddressSanitizer and
    UndefinedBehaviorSanitizer, into _build/librbd_hostsan.so."""
    os.makedirs(os.path.dirname(SANITIZED_LIB), exist_ok=True)
    tmp = SANITIZED_LIB + ".tmp"
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + ["-O1"] + SANITIZER_FLAGS
    cmd = [hipcc(), *flags, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    os.replace(tmp, SANITIZED_LIB)
    return SANITIZED_LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
