"""The host runtime's validation paths under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only; the kernel side is a test double, tests/sanitize_launch_double.cpp).  The driver,
tests/sanitize_host_paths.cpp, refuses every malformed description, stream and argument through
the C ABI and reads the error messages; any sanitizer report or failed check fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# host-only sanitizers: each option applies to the host compilation alone
SANITIZE = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=undefined".split()


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is not installed")
def test_host_runtime_validation_paths_are_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_paths")
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer"] + SANITIZE + [
        "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2006_07478_amd", "csrc"),
        os.path.join(ROOT, "paper_2006_07478_amd", "csrc", "rs_runtime.cpp"),
        os.path.join(ROOT, "tests", "sanitize_launch_double.cpp"),
        os.path.join(ROOT, "tests", "sanitize_host_paths.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stdout + b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "cpu"], capture_output=True, text=True, timeout=120, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
    assert "0 failed checks" in out
