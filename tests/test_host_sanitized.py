"""The library's host code (argument checks, launch plans, workspace layout,
batch plans) under AddressSanitizer and UndefinedBehaviorSanitizer: the
C-ABI checks of test_abi_cpu.py run, in a child process, against a build whose
host code is instrumented (device code built as usual), with the sanitizer
runtime preloaded and every report fatal."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_checks_under_asan_and_ubsan():
    from paper_1503_05947_amd import _build
    lib = _build.build_host_sanitized()
    rt = _build.asan_runtime()
    env = dict(os.environ)
    env["RBD_LIBRARY"] = lib
    env["LD_PRELOAD"] = rt + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["LD_LIBRARY_PATH"] = os.path.dirname(rt) + (":" + env["LD_LIBRARY_PATH"] if env.get("LD_LIBRARY_PATH") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
