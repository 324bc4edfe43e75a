"""Host C/C++ under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle and the seeded generator (tests/host_sanitize_selftest.c) and the
serving engine's HBM-budget allocator (tests/arena_selftest.cpp), built with
gcc / g++ on the CPU.  Skipped where the toolchain has no sanitizer runtime."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _have_sanitizers(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", *SAN, "-o", str(tmp_path / "probe"), str(src)], capture_output=True)
    return r.returncode == 0


def test_oracle_and_generator_sanitized(tmp_path):
    if not _have_sanitizers(tmp_path):
        pytest.skip("gcc has no sanitizer runtime here")
    exe = tmp_path / "host_sanitize"
    subprocess.run(["gcc", "-std=c11", *SAN, "-ffp-contract=off", "-o", str(exe),
                    os.path.join(ROOT, "tests", "host_sanitize_selftest.c"),
                    os.path.join(ROOT, "oracle", "rbsm_oracle.c"),
                    os.path.join(ROOT, "synth", "synth.c"), "-lm"], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, env=ENV).stdout
    assert "host sanitize ok" in out


def test_arena_sanitized(tmp_path):
    if not _have_sanitizers(tmp_path):
        pytest.skip("g++ has no sanitizer runtime here")
    exe = tmp_path / "arena_selftest"
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_1711_07793_amd", "csrc"),
                    "-o", str(exe), os.path.join(ROOT, "tests", "arena_selftest.cpp")], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, env=ENV).stdout
    assert "arena ok" in out
