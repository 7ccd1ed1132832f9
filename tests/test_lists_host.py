"""Host emulation of the per-tile target-list enumeration (CPU only, no GPU).

Compiles tests/list_emul.cpp against the library's own list-geometry header
(the functions the device count, fill and check kernels call) for the host
and runs it: on edge-case geometries every target of every slice must be
enumerated exactly once, in the tile and border class its coordinates give."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_list_enumeration_edge_geometries():
    out = os.path.join(ROOT, "_build", "list_emul")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = [HIPCC, "--offload-host-only", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2511_01893_amd", "csrc"), os.path.join(ROOT, "tests", "list_emul.cpp"),
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([out], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count("each listed once") == 10
