"""The serving engine's HBM-budget allocator (csrc/arena.hpp), built with g++
and checked on the CPU against a byte-map model."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_selftest(tmp_path):
    exe = tmp_path / "arena_selftest"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "paper_1711_07793_amd", "csrc"),
                    "-o", str(exe), os.path.join(ROOT, "tests", "arena_selftest.cpp")], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    assert "arena ok" in out
