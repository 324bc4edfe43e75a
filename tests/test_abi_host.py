"""Host-only checks of the C ABI library: it loads, exports every symbol the
header declares, and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbsm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                                 text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_1711_07793_amd as rb
    if not os.path.exists(rb.LIB_PATH):
        from paper_1711_07793_amd import build
        build.build()
    return rb.load_library()


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for want in ("rbsm_visibility", "rsmss_visibility", "sm_visibility", "rbsm_footprint",
                 "rbsm_last_error", "rbsm_abi_version", "rbsm_pass_tuned", "rbsm_default_tuning",
                 "rbsm_plan_create", "rbsm_plan_launch", "rbsm_plan_update", "rbsm_plan_autotune",
                 "rbsm_plan_capture", "rbsm_plan_destroy"):
        assert want in names, names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_abi_version(lib):
    assert lib.rbsm_abi_version() == 103


def _p(**kw):
    import paper_1711_07793_amd as rb
    base = dict(width=64, height=64, pitch=64, depth_bias=0.0, max_dist=16, kernel_radius=0, view_width=0)
    base.update(kw)
    return rb.RbsmParams(**base)


@pytest.mark.parametrize("bad", [
    dict(width=0), dict(height=0), dict(width=70000), dict(pitch=10), dict(max_dist=0),
    dict(max_dist=65), dict(kernel_radius=-1), dict(kernel_radius=33), dict(view_width=-1)])
def test_invalid_params_rejected_on_host(lib, bad):
    p = _p(**bad)
    # fake, never dereferenced device addresses: validation fails first
    st = lib.rsmss_visibility(0x1000, 0x100000, 16, ctypes.byref(p), 0x200000, None)
    assert st == -1
    assert lib.rbsm_last_error().decode().startswith("rsmss_visibility:")


def test_hard_rejects_radius_and_nulls(lib):
    p = _p(kernel_radius=1)
    assert lib.rbsm_visibility(0x1000, 0x100000, 16, ctypes.byref(p), 0x200000, None) == -1
    p = _p()
    assert lib.rbsm_visibility(0, 0x100000, 16, ctypes.byref(p), 0x200000, None) == -1
    assert lib.rbsm_visibility(0x1000, 0x100000, 16, None, 0x200000, None) == -1
    assert lib.rbsm_visibility(0x1000, 0x100000, -1, ctypes.byref(p), 0x200000, None) == -1
    assert "null" in lib.rbsm_last_error().decode() or "n < 0" in lib.rbsm_last_error().decode()


def test_overlapping_output_rejected(lib):
    p = _p()
    frags = 0x100000
    assert lib.rbsm_visibility(0x1000000, frags, 16, ctypes.byref(p), frags + 8, None) == -1
    assert "overlap" in lib.rbsm_last_error().decode()


def test_empty_call_is_a_noop(lib):
    p = _p()
    assert lib.rbsm_visibility(0, 0, 0, ctypes.byref(p), 0, None) == 0
    assert lib.rsmss_visibility(0, 0, 0, ctypes.byref(p), 0, None) == 0


def test_footprint_mode_checked(lib):
    p = _p()
    assert lib.rbsm_footprint(0x1000, 0x100000, 4, ctypes.byref(p), 7, 0x200000, None) == -1


def test_tuning_validated_on_host(lib):
    import paper_1711_07793_amd as rb
    d = lib.rbsm_default_tuning()
    assert d.tile_w in (16, 32, 64) and d.apron >= 1 and d.lds_cap >= 256
    p = _p()
    for bad in (rb.RbsmTuning(24, 1, 4096), rb.RbsmTuning(32, 0, 4096), rb.RbsmTuning(32, 1, 100000),
                rb.RbsmTuning(32, 1, 2048, 2, 0, 0), rb.RbsmTuning(32, 1, 2048, 0, 3, 0),
                rb.RbsmTuning(32, 1, 2048, 0, 0, 5), rb.RbsmTuning(32, 1, 2048, 1, 4, 8),
                rb.RbsmTuning(32, 1, 2048, 0, 0, 0, 13), rb.RbsmTuning(32, 1, 2048, 0, 0, 0, -2),
                # persistent launches take the default walk blocking only
                rb.RbsmTuning(32, 1, 2048, 1, 1, 4), rb.RbsmTuning(32, 1, 2048, 1, 2, 8)):
        assert lib.rbsm_pass_tuned(0, 0x1000, 0x100000, 16, ctypes.byref(p), ctypes.byref(bad), 0x200000, None) == -1
    assert lib.rbsm_pass_tuned(3, 0x1000, 0x100000, 16, ctypes.byref(p), ctypes.byref(d), 0x200000, None) == -1
    h = ctypes.c_void_p()
    jobs = (rb.RbsmJob * 1)()
    jobs[0] = rb.RbsmJob(0x1000000, 0x2000000, 64, p, 0, 0x3000000)
    bad = rb.RbsmTuning(64, 1, 2048, 1, 4, 4)
    assert lib.rbsm_plan_create(jobs, 1, ctypes.byref(bad), ctypes.byref(h)) == -1 and not h.value
    assert "tuning" in lib.rbsm_last_error().decode()


def test_plan_rejects_bad_jobs_on_host(lib):
    import paper_1711_07793_amd as rb
    h = ctypes.c_void_p()
    p = _p()
    jobs = (rb.RbsmJob * 2)()
    jobs[0] = rb.RbsmJob(0x1000000, 0x2000000, 64, p, 0, 0x3000000)
    jobs[1] = rb.RbsmJob(0x1000000, 0x2000000, 64, p, 5, 0x3100000)  # bad mode
    assert lib.rbsm_plan_create(jobs, 2, None, ctypes.byref(h)) == -1 and not h.value
    jobs[1] = rb.RbsmJob(0x1000000, 0x2000000, 64, p, 0, 0x3000010)  # outputs overlap
    assert lib.rbsm_plan_create(jobs, 2, None, ctypes.byref(h)) == -1
    assert "overlap" in lib.rbsm_last_error().decode()
    q = _p(kernel_radius=2)
    jobs[1] = rb.RbsmJob(0x1000000, 0x2000000, 64, q, 0, 0x3100000)  # a radius on a hard job
    assert lib.rbsm_plan_create(jobs, 2, None, ctypes.byref(h)) == -1
    assert "kernel_radius" in lib.rbsm_last_error().decode()
    assert lib.rbsm_plan_create(jobs, 0, None, ctypes.byref(h)) == -1
    assert lib.rbsm_plan_launch(None, None) == -1
    assert lib.rbsm_plan_fragments(None) == -1


def test_composite_validated_on_host(lib):
    vp = ctypes.c_void_p
    ptrs = (vp * 2)(0x100000, 0x200000)
    modes = (ctypes.c_int32 * 2)(0, 1)
    w = (ctypes.c_float * 2)(0.5, 0.5)
    assert lib.rbsm_composite(16, 0, ptrs, modes, w, 0x300000, None) == -1      # no lights
    assert lib.rbsm_composite(16, 9, ptrs, modes, w, 0x300000, None) == -1      # too many
    assert lib.rbsm_composite(-1, 2, ptrs, modes, w, 0x300000, None) == -1
    assert lib.rbsm_composite(16, 2, None, modes, w, 0x300000, None) == -1
    bad = (ctypes.c_int32 * 2)(0, 3)
    assert lib.rbsm_composite(16, 2, ptrs, bad, w, 0x300000, None) == -1
    assert lib.rbsm_composite(16, 2, ptrs, modes, w, 0x200008, None) == -1      # out overlaps an input
    assert "overlap" in lib.rbsm_last_error().decode()
    assert lib.rbsm_composite(0, 2, ptrs, modes, w, 0, None) == 0               # empty is a no-op


def test_engine_arguments_validated_on_host(lib):
    import paper_1711_07793_amd as rb
    h = ctypes.c_void_p()
    assert lib.rbsm_engine_create(100, 4, ctypes.byref(h)) == -1 and not h.value   # budget too small
    assert lib.rbsm_engine_create(1 << 20, 0, ctypes.byref(h)) == -1
    assert lib.rbsm_engine_create(1 << 20, 4, None) == -1
    t = ctypes.c_int64()
    q = rb.RbsmRequest()
    assert lib.rbsm_engine_submit(None, ctypes.byref(q), ctypes.byref(t)) == -1
    lid = ctypes.c_int32()
    assert lib.rbsm_engine_add_light(None, 0x1000, 4, 4, 4, ctypes.byref(lid)) == -1
    assert lib.rbsm_engine_wait(None, 1, 0, None) == -1
    assert lib.rbsm_engine_get_stats(None, None) == -1
    lib.rbsm_engine_destroy(None)


def test_rasterize_validated_on_host(lib):
    d = ctypes.c_double
    args = lambda **k: dict(dict(prims=0x100000, n=4, W=64, H=64, pitch=64, out=0x200000), **k)
    def call(a):
        return lib.rbsm_rasterize(a["prims"], a["n"], d(0.9), d(0.0), d(0.0), a["W"], a["H"], a["pitch"], a["out"],
                                  None)
    assert call(args(W=0)) == -1
    assert call(args(H=70000)) == -1
    assert call(args(pitch=10)) == -1
    assert call(args(n=-1)) == -1
    assert call(args(out=0)) == -1
    assert call(args(prims=0)) == -1
    assert call(args(out=0x100000 + 64)) == -1             # map over the primitive records
    assert "overlap" in lib.rbsm_last_error().decode()


def test_tune_cache_file_round_trip(lib, tmp_path):
    """The autotuner cache is host state: loading, saving and clearing it
    touch no GPU."""
    import paper_1711_07793_amd as rb
    rb.tune_cache_clear()
    src = tmp_path / "tune.txt"
    src.write_text("# comment\n"
                   "gfx950-cu256/00000000deadbeef 64 1 2048 1 2 4 -1\n"
                   "gfx950-cu256/0123456789abcdef 32 2 3072 0 2 4 5\n")
    assert rb.tune_cache_load(str(src)) == 2
    out = tmp_path / "saved.txt"
    rb.tune_cache_save(str(out))
    lines = sorted(l for l in out.read_text().splitlines() if not l.startswith("#"))
    assert lines == ["gfx950-cu256/00000000deadbeef 64 1 2048 1 2 4 -1",
                     "gfx950-cu256/0123456789abcdef 32 2 3072 0 2 4 5"]
    rb.tune_cache_clear()
    rb.tune_cache_save(str(out))
    assert [l for l in out.read_text().splitlines() if not l.startswith("#")] == []


@pytest.mark.parametrize("line", ["key 24 1 2048 0 2 4 -1", "key 32 1 2048 0 3 4 -1", "key 32 1 2048 2 2 4 -1",
                                  "key 32 1", "key 32 9 2048 0 2 4 -1", "key 32 1 2048 0 2 4 13",
                                  "key 32 1 2048 0 2 4"])
def test_tune_cache_rejects_bad_entries(lib, tmp_path, line):
    import paper_1711_07793_amd as rb
    f = tmp_path / "bad.txt"
    f.write_text(line + "\n")
    with pytest.raises(rb.RbsmError):
        rb.tune_cache_load(str(f))
    with pytest.raises(rb.RbsmError):
        rb.tune_cache_load(str(tmp_path / "missing.txt"))
    rb.tune_cache_clear()


def test_noalloc_batch_rejects_oversized_requests_on_host(lib):
    """The allocation-free entry point's limits (4096 jobs, 1,916,928 tiles)
    and its argument checks come before any GPU call."""
    import paper_1711_07793_amd as rb
    p = _p(view_width=64)
    jobs = (rb.RbsmJob * 4097)()
    for k in range(4097):
        jobs[k] = rb.RbsmJob(0x1000000, 0x2000000, 64, p, 0, 0x10000000 + 256 * k)
    assert lib.rbsm_batch_launch_noalloc(jobs, 4097, None, None) == -1
    assert "4096" in lib.rbsm_last_error().decode()
    big = (rb.RbsmJob * 1)()
    n = 1024 * 1916929  # one tile more than the table holds (flat 1024-fragment tiles)
    big[0] = rb.RbsmJob(0x1000000, 0x20000000000, n, _p(), 0, 0x40000000000)
    assert lib.rbsm_batch_launch_noalloc(big, 1, None, None) == -1
    assert "tiles" in lib.rbsm_last_error().decode()
    bad = (rb.RbsmJob * 1)()
    bad[0] = rb.RbsmJob(0x1000000, 0x2000000, 64, p, 3, 0x3000000)
    assert lib.rbsm_batch_launch_noalloc(bad, 1, None, None) == -1
    t = rb.RbsmTuning(24, 1, 2048)
    assert lib.rbsm_batch_launch_noalloc(jobs, 1, ctypes.byref(t), None) == -1
