"""The C ABI's host code under AddressSanitizer and UBSan (CPU only, no GPU).

Builds liblam's host code alone (host-only compilation: no device code, so nothing can be launched)
with both sanitizers, links tests/abi_host.cpp against it with the same sanitizers, and runs it: plan
construction on power-of-two and 3 2^k sizes and every half-width, the validation and state errors
of every entry point, the memoization layout, and the ADMM-Offload planner on 400 random
timelines.  Any out-of-bounds access, use after free or undefined behaviour aborts the driver."""
import os
import subprocess

import pytest

from paper_2511_01893_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ of the ROCm toolchain not found")
def test_abi_host_code_under_asan_ubsan():
    lib = B.build_host_sanitized()
    exe = os.path.join(ROOT, "_build", "abi_host")
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_host.cpp"),
           lib, "-Wl,-rpath," + os.path.dirname(lib), "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi host checks ok" in r.stdout
