"""The host-side plan construction (CPU C++) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run over the supported parameter range: no
memory error, no undefined behaviour, and the node-table invariants hold."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1409_2014_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_plan_construction_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "plan_host_driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROOT}/include", f"-I{CSRC}", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "host", "plan_host_driver.cpp"), os.path.join(CSRC, "plan_host.cpp"),
           "-o", str(exe)]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-2000:]
    # the sanitizer runtime may not be first in the load order when the
    # environment preloads a library: let it run anyway
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-2000:])
    assert "runtime error" not in run.stderr
    assert run.stdout.strip().startswith("OK")
