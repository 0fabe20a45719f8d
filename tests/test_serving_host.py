"""Host logic of the serving layer, on the CPU: the pool allocator that admits
jobs by memory (first fit, no overlap, full coalescing)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pool_allocator(tmp_path):
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-I",
                    os.path.join(ROOT, "paper_2609_02876_amd", "csrc"),
                    os.path.join(ROOT, "tests", "arena_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"
