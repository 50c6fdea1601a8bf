"""The host planner (sampling resolution, backed-row checks, flow plans and
chunking) built with g++ alone under AddressSanitizer and
UndefinedBehaviorSanitizer, driven through valid, adversarial (overflowing
strides, absurd row counts) and invalid specs (CPU only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_07339_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "plan_sanitize")
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    cmd = (["g++", "-std=c++17", "-O1", "-g"] + flags +
           ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
            os.path.join(ROOT, "tests", "native", "plan_sanitize.cpp"),
            os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "flow_plan.cpp"), "-o", exe])
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok: 0 failure(s)" in r.stdout
