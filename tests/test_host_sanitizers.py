"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the option validation, cluster tree, level schedule and structure query of
csrc/plan.cpp are compiled with g++ -fsanitize=address,undefined together with
tests/sanitize_driver.cpp and run; any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

from paper_1701_00182_amd import build as b

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which(b.CXX) is None, reason="no host C++ compiler")
def test_plan_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    cmd = ([b.CXX] + b.host_flags() + ["-O1", "-g", "-fno-omit-frame-pointer",
                                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                        os.path.join(b.CSRC, "plan.cpp"), os.path.join(HERE, "sanitize_driver.cpp"),
                                        "-o", exe])
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "all checks passed" in r.stdout
