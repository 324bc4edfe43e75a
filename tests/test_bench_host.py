"""Host-side checks of bench.py: the kernel-source hash that keys the
committed traffic figures, the lookup of those figures, and the one-GPU
refusal."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNED = {"tile_w": 32, "apron": 1, "lds_cap": 2048, "persistent": 0, "walk_first": 2, "walk_block": 4,
         "xcd_chunk": 3}


def test_code_tokens_ignore_comments_and_spacing_only():
    a = "int f(int x) {\n    return x + 1;  // one more\n}\n"
    b = "/* doc */ int f(int x) { return x + 1; }"
    c = "int f(int x) { return x + 2; }"
    assert bench.code_tokens(a) == bench.code_tokens(b)
    assert bench.code_tokens(a) != bench.code_tokens(c)
    assert bench.code_tokens("a/*x\ny*/b") == "a b"


def test_traffic_figures_match_the_current_kernel():
    """The committed summary was taken on the current kernel code and holds
    the tuning the autotuner settles on for the headline."""
    h = bench.kernel_source_hash()
    got = bench.read_traffic(h, TUNED)
    assert got is not None and got > 1.0e9
    assert bench.read_traffic("0" * 16, TUNED) is None
    assert bench.read_traffic(h, dict(TUNED, tile_w=16)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0 and "one GPU" in r.stdout + r.stderr
