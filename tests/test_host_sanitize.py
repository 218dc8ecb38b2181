"""The library's host side (argument validation and the FP64 plan builder,
paper_2411_17804_amd/csrc/host.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer by the host compiler and run on the CPU: any
out-of-bounds access, leak or undefined behaviour aborts the driver."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_17804_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_side_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "host_sanitize")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-I", "/opt/rocm/include",
               os.path.join(CSRC, "host.cpp"), os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"),
               "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
        assert "host checks OK" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_the_sanitizer_build_catches_an_out_of_bounds_read():
    # the same flags on a program that reads one element past a heap array:
    # the run must fail, so a passing driver above means something
    src = "#include <vector>\nint main(int c, char **){ std::vector<int> v(4, 1); return v.data()[3 + c]; }\n"
    with tempfile.TemporaryDirectory() as d:
        path, exe = os.path.join(d, "oob.cpp"), os.path.join(d, "oob")
        open(path, "w").write(src)
        r = subprocess.run(["g++", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                            path, "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:verify_asan_link_order=0")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=60)
        assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
