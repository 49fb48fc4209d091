"""The host geometry code (CSR builder, radial codes, row schedule) built
with AddressSanitizer and UndefinedBehaviorSanitizer and run over small,
odd, masked, off-centre and extreme geometries (CPU only): no sanitizer
report, and every property checked by ``sanitize/geometry_check.cpp``
holds (exact row bounds, sorted rows, coefficients summing to one, masked
pixels absent, the schedule a permutation of the bins, error codes)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIP_INCLUDE = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(HIP_INCLUDE),
                    reason="needs g++ and the HIP headers")
def test_geometry_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "geometry_check"
    # host code only: the HIP headers are read for the stream type, with the
    # platform macro that hipcc itself defines for host compilation
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-static-libasan",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", HIP_INCLUDE,
           os.path.join(ROOT, "paper_2411_09515_amd", "csrc", "geometry.cpp"),
           os.path.join(HERE, "sanitize", "geometry_check.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "geometry checks ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
