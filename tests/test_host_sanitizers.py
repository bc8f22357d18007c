"""The library's host C++ built with AddressSanitizer and UndefinedBehaviorSanitizer
on the CPU (g++ only, no device code): the FC-Gram tables in binary128 and the
matching stencils' star placement, node selection and weights, driven by
tests/host_check.cpp on the unit disc; the stencils come out byte-identical with one
and with three threads."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2010_03901_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    cmd = ["g++", "-O1", "-g", "-std=gnu++17", "-ffp-contract=off", "-fno-builtin-sin", "-fno-builtin-cos",
           "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
           os.path.join(HERE, "host_check.cpp"), os.path.join(CSRC, "matching_host.cpp"),
           os.path.join(CSRC, "fcgram_quad.cpp"), "-lquadmath", "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-4000:]
    digests = []
    for threads in ("1", "3"):   # the parallel loops write every entry whatever the thread count
        env = dict(os.environ, OMP_NUM_THREADS=threads, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=600)
        assert r.returncode == 0 and "HOST_CHECK_OK" in r.stdout, r.stdout[-4000:]
        digests.append([l for l in r.stdout.splitlines() if l.startswith("stencil digest")])
    assert digests[0] and digests[0] == digests[1], digests
