"""The host construction and FP64 executor built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, no GPU code) and run over both readings,
both super-leaf sizes, both storage dtypes' schedules and a two-curve
layout (tests/asan/host_checks.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_construction_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    src = os.path.join(ROOT, "paper_1901_11371_amd", "csrc")
    exe = str(tmp_path / "host_checks")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
           os.path.join(ROOT, "tests", "asan", "host_checks.cpp"), os.path.join(src, "plan.cpp"),
           os.path.join(src, "schedule.cpp"), os.path.join(src, "hankel.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "all host checks passed" in r.stdout
