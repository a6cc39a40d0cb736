"""Build libbk_san.so: the same sources with AddressSanitizer and
UndefinedBehaviorSanitizer in the HOST code only (the gfx950 device code is
compiled as usual), for the host-side argument, size and workspace checks of
the C ABI.  The GPU never runs it.

Usage: python -m paper_1504_05477_amd.build_sanitized
Load it with the clang ASan runtime preloaded (SAN_RUNTIME below)."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

from . import build as b

SAN_BUILD = os.path.join(b.BUILD, "san")
# kept with the build objects: a test artefact, not part of the package
SAN_LIB = os.path.join(SAN_BUILD, "libbk_san.so")
# every sanitizer flag applies to the host pass only
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def runtime() -> str | None:
    """The clang ASan runtime of the ROCm toolchain (to LD_PRELOAD)."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _compile(src: str) -> str:
    obj = os.path.join(SAN_BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [b.HIPCC, *b.COMMON, "-O1", "-g", *SAN_FLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(SAN_BUILD, exist_ok=True)
    srcs = b.sources()
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = SAN_LIB + ".tmp"
    cmd = [b.HIPCC, f"--offload-arch={b.ARCH}", "-shared", "-fPIC", *SAN_FLAGS, *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, SAN_LIB)
    if verbose:
        print(f"built {SAN_LIB}")
    return SAN_LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
