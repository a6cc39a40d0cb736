"""The host-side C ABI checks (tests/test_abi.py: argument rules, workspace
sizes, BK_EINVAL / BK_ENOMEM before any launch) run again against the build
whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer
(paper_1504_05477_amd/build_sanitized.py), in a child process with the clang
ASan runtime preloaded.  Any sanitizer report makes the child fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_checks_under_asan_ubsan():
    from paper_1504_05477_amd import build_sanitized as bs
    rt = bs.runtime()
    if rt is None:
        pytest.skip("no clang ASan runtime in this toolchain")
    if not os.path.exists(bs.SAN_LIB):
        pytest.skip("libbk_san.so not built (python -m paper_1504_05477_amd.build_sanitized)")
    env = dict(os.environ)
    env.update({"BK_LIBRARY": bs.SAN_LIB, "LD_PRELOAD": rt,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=23",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=24"})
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (res.stdout + res.stderr)[-3000:]
    assert res.returncode == 0, tail
    assert "AddressSanitizer" not in tail and "runtime error" not in tail, tail
