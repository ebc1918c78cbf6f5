"""Host-code AddressSanitizer / UndefinedBehaviorSanitizer build of the
library, for the CPU test of its argument validation and host logic.

Each translation unit is compiled as for the library, with the sanitizers
on the host side only (-Xarch_host: the device code is built as usual, never
with a sanitizer), linked into _build/sanitize/libfurax_san.so together with
the HIP runtime, and a C++ driver (tests/host_abi_check.cpp) is linked against
it with the same sanitizers.  Every call the driver makes returns before any
device work.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

from . import build as _b

OUT = os.path.join(_b.ROOT, "_build", "sanitize")
LLVM = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin")
CLANGXX = os.path.join(LLVM, "clang++") if os.path.exists(os.path.join(LLVM, "clang++")) \
    else shutil.which("clang++")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
SAN_LINK = ["-fsanitize=address,undefined", "-shared-libasan"]


def _asan_runtime_dir() -> str:
    """Directory of the compiler's shared ASan runtime (for the rpath)."""
    r = subprocess.run([CLANGXX, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return os.path.dirname(path)
    rt = subprocess.run([CLANGXX, "-print-resource-dir"], capture_output=True, text=True)
    return os.path.join(rt.stdout.strip(), "lib", "linux")


def _compile(src: str) -> str:
    obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    cmd = [_b.HIPCC, *_b.FLAGS, *SAN_HOST, "-g", "-c",
           os.path.join(_b.CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitized compile failed for {src}:\n{r.stderr}")
    return obj


def build() -> str:
    """Build the sanitized library and the driver; returns the driver's path."""
    os.makedirs(OUT, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(_b.SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, _b.SOURCES))
    lib = os.path.join(OUT, "libfurax_san.so")
    rocm_lib = _b.ROCM_LIB
    rt = _asan_runtime_dir()
    cmd = [CLANGXX, "-shared", *SAN_LINK, f"-Wl,-rpath,{rt}", *objs, f"-L{rocm_lib}", f"-Wl,-rpath,{rocm_lib}",
           "-lamdhip64", "-lrocprofiler-sdk-roctx", "-o", lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitized link failed:\n{r.stderr}")
    exe = os.path.join(OUT, "host_abi_check")
    drv = os.path.join(_b.ROOT, "tests", "host_abi_check.cpp")
    cmd = [CLANGXX, "-std=c++17", "-g", "-D__HIP_PLATFORM_AMD__", *SAN_LINK, f"-Wl,-rpath,{rt}",
           f"-I{_b.INCLUDE}",
           f"-I{os.path.join(os.path.dirname(rocm_lib), 'include')}", drv, f"-L{OUT}",
           f"-Wl,-rpath,{OUT}", "-lfurax_san", f"-L{rocm_lib}", f"-Wl,-rpath,{rocm_lib}",
           "-lamdhip64", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver build failed:\n{r.stderr}")
    return exe
