"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library's host-only numerics (tridiagonal QL and sign(T) e_1, the Hermitian
Jacobi eigensolver, the Zolotarev coefficients) are built with g++ and both
sanitizers into a standalone driver (``host_sanitize_main.cpp``) that checks its
own results; any sanitizer report aborts it with a non-zero status.  The HIP
sources are not part of this build: their host parts need the HIP runtime.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not on PATH")
def test_host_numerics_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "host_sanitize_main.cpp"),
           os.path.join(ROOT, "paper_1410_7170_amd", "csrc", "zolotarev.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ)
    # leak checking needs ptrace, which a container may not allow; the
    # address and undefined-behaviour checks do not
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout + r.stderr
    assert "runtime error" not in r.stderr, r.stderr
