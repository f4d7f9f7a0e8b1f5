"""Host-side logic of the library, on the CPU (no GPU, no HIP runtime)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_server_arena_allocator(tmp_path):
    exe = tmp_path / "arena_test"
    src = os.path.join(ROOT, "tests", "host", "arena_test.cpp")
    inc = os.path.join(ROOT, "paper_2106_00454_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Xlinker", "--no-as-needed", "-I", inc, src, "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "arena ok" in r.stdout
