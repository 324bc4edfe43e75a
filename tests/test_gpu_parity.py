"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: hard masks bit-equal except on at most 1e-5 of the fragments, each of
which must lie within 1e-6 of a decision boundary (binary64 margin from the
oracle); RSMSS / RPCF values within 1e-5 absolute; read-set bitmaps bit-equal.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

HARD_FRAC = 1e-5
MARGIN = 1e-6
SOFT_TOL = 1e-5


@pytest.fixture(scope="module")
def rb():
    import paper_1711_07793_amd as rb
    rb.load_library()
    assert torch.cuda.is_available()
    return rb


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_hard(map_np, frags_np, params, got):
    want = oracle.rbsm_hard(map_np, frags_np, params)
    bad = np.nonzero(got != want)[0]
    assert len(bad) <= max(0, int(HARD_FRAC * len(want))), f"{len(bad)} of {len(want)} differ"
    for k in bad:
        assert oracle.margin(map_np, frags_np[k], params, True) < MARGIN, k


def check_soft(map_np, frags_np, params, got, idx=None):
    if idx is None:
        want = oracle.rsmss(map_np, frags_np, params)
    else:
        want = oracle.rsmss(map_np, frags_np[idx], params)
        got = got[idx]
    err = np.abs(got.astype(np.float64) - want.astype(np.float64))
    assert err.max(initial=0.0) <= SOFT_TOL, (err.max(), np.argmax(err))


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("cfg,small", [(1, False), (2, True), (2, False), (3, True)])
def test_hard_workloads(rb, cfg, small):
    c = synth.make_config(cfg, 1000 * cfg + 1, small=small)
    say(f"hard cfg{cfg} small={small} n={len(c['frags'])}")
    p = dict(c["params"], kernel_radius=0)
    got = rb.rbsm_visibility(dev(c["map"]), dev(c["frags"]), p).cpu().numpy()
    check_hard(c["map"], c["frags"], p, got)


@pytest.mark.parametrize("cfg,small", [(1, False), (2, True), (3, True), (3, False)])
def test_rsmss_workloads(rb, cfg, small):
    c = synth.make_config(cfg, 1000 * cfg + 2, small=small)
    say(f"rsmss cfg{cfg} small={small} n={len(c['frags'])}")
    p = dict(c["params"], kernel_radius=0)
    got = rb.rsmss_visibility(dev(c["map"]), dev(c["frags"]), p).cpu().numpy()
    check_soft(c["map"], c["frags"], p, got)


def test_rpcf_small_frame_every_seventh_fragment(rb):
    c = synth.make_config(3, 3003, small=True)
    r = c["light_radius"]
    say(f"rpcf small r={r}")
    p = dict(c["params"], kernel_radius=r)
    got = rb.rsmss_visibility(dev(c["map"]), dev(c["frags"]), p).cpu().numpy()
    idx = np.arange(0, len(got), 7)
    check_soft(c["map"], c["frags"], p, got, idx)
    assert np.all((got >= 0) & (got <= 1))


def test_rpcf_full_size_sampled(rb):
    c = synth.make_config(3, 3001)
    r = c["light_radius"]
    say(f"rpcf full r={r} n={len(c['frags'])}")
    p = dict(c["params"], kernel_radius=r)
    got = rb.rsmss_visibility(dev(c["map"]), dev(c["frags"]), p).cpu().numpy()
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(len(got), 1500, replace=False))
    check_soft(c["map"], c["frags"], p, got, idx)


@pytest.mark.parametrize("r,max_dist", [(1, 1), (1, 16), (3, 16), (7, 16), (9, 16), (10, 16), (12, 64), (15, 16),
                                        (2, 29), (30, 1), (2, 40), (6, 64), (31, 4), (32, 2)])
def test_rpcf_radii_and_reach(rb, r, max_dist):
    """Every RPCF route: staged bands (screen tiles; up to r = 9 with the
    transposed band, beyond it the row band alone), reads from global memory
    (bands too large), and the per-term form when a column of 2r+3 rows no
    longer fits one word (r > 30)."""
    c = synth.make_config(3, 3005, small=True)
    n = len(c["frags"])
    idx = np.arange(0, n, max(1, n // (4000 if r <= 7 else (800 if r <= 15 else 200))))
    p = dict(c["params"], kernel_radius=r, max_dist=max_dist)
    say(f"rpcf r={r} maxd={max_dist} n={n}")
    got = rb.rsmss_visibility(dev(c["map"]), dev(c["frags"]), p).cpu().numpy()
    check_soft(c["map"], c["frags"], p, got, idx)
    assert np.all((got >= 0) & (got <= 1))


@pytest.mark.parametrize("vw", [0, 97])
def test_rpcf_flat_and_scattered_fragments(rb, vw):
    """Uniform random fragments: tile boxes are far larger than LDS, so words
    come from global memory; view_width 97 makes ragged 2-D tiles."""
    c = synth.make_config(1, 1009, small=True)
    f = np.ascontiguousarray(c["frags"][:6001])
    for r in (1, 4):
        p = dict(c["params"], kernel_radius=r, view_width=vw)
        got = rb.rsmss_visibility(dev(c["map"]), dev(f), p).cpu().numpy()
        check_soft(c["map"], f, p, got)


def test_rpcf_clamped_edges_of_tiny_maps(rb):
    """Boxes that hang over every map border (clamp-to-edge reads)."""
    rng = np.random.default_rng(8)
    for (H, W) in [(1, 1), (3, 2), (9, 17), (40, 33)]:
        m = np.where(rng.random((H, W)) < 0.4, 0.5, 0.9).astype(np.float32)
        f = _frags_for(W, H, 3000 + W, seed=W, spill=0.2)
        for r, vw in ((2, 0), (5, 50), (11, 50)):
            p = dict(width=W, height=H, pitch=W, depth_bias=1e-4, max_dist=12, kernel_radius=r, view_width=vw)
            got = rb.rsmss_visibility(dev(m), dev(f), p).cpu().numpy()
            check_soft(m, f, p, got)


@pytest.mark.parametrize("mode", [0, 1])
def test_footprint_matches_oracle_reads(rb, mode):
    c = synth.make_config(2, 2001, small=True)
    p = dict(c["params"], kernel_radius=0)
    got = rb.rbsm_footprint(dev(c["map"]), dev(c["frags"]), p, mode).cpu().numpy()
    want, _ = oracle.touched_texels(c["map"], c["frags"], p, hard=(mode == 0))
    assert np.array_equal(got, want)


def test_plain_sm(rb):
    c = synth.make_config(2, 2001, small=True)
    got = rb.sm_visibility(dev(c["map"]), dev(c["frags"]), c["params"]).cpu().numpy()
    assert np.array_equal(got, oracle.shadow_map(c["map"], c["frags"], c["params"]))


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def _adversarial_maps():
    rng = np.random.default_rng(77)
    maps = {}
    W = 96
    ii, jj = np.meshgrid(np.arange(W), np.arange(W))
    maps["checker"] = np.where((ii + jj) % 2 == 0, 0.5, 0.9).astype(np.float32)
    maps["checker2"] = np.where(((ii // 2) + (jj // 3)) % 2 == 0, 0.5, 0.9).astype(np.float32)
    bars = np.full((W, W), 0.9, np.float32)
    bars[:, ::5] = 0.5
    bars[::7, :] = 0.5
    maps["bars"] = bars
    border = np.full((W, W), 0.9, np.float32)
    border[0, :] = 0.5
    border[:, -1] = 0.5
    border[40:60, 0:3] = 0.5
    maps["border"] = border
    noise = np.where(rng.random((W, W)) < 0.4, 0.5, 0.9).astype(np.float32)
    maps["noise"] = noise
    depths = rng.choice(np.array([0.3, 0.5, 0.7, 0.9], np.float32), (W, W))
    maps["multidepth"] = depths
    return maps


def _frags_for(W, H, n, seed, spill=0.0):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-spill, 1 + spill, n)
    v = rng.uniform(-spill, 1 + spill, n)
    z = rng.choice(np.array([0.4, 0.6, 0.8, 0.9], np.float32), n)
    return np.stack([u, v, z], 1).astype(np.float32)


@pytest.mark.parametrize("name", list(_adversarial_maps().keys()))
@pytest.mark.parametrize("max_dist", [1, 3, 16, 64])
def test_adversarial_maps(rb, name, max_dist):
    m = _adversarial_maps()[name]
    H, W = m.shape
    f = _frags_for(W, H, 40000 + 37, seed=max_dist, spill=0.05)
    p = dict(width=W, height=H, pitch=W, depth_bias=1e-4, max_dist=max_dist, kernel_radius=0)
    md, fd = dev(m), dev(f)
    check_hard(m, f, p, rb.rbsm_visibility(md, fd, p).cpu().numpy())
    check_soft(m, f, p, rb.rsmss_visibility(md, fd, p).cpu().numpy())


def _screen_frags(W, H, vw, vh, seed, spill=0.05):
    """Fragments of a vw x vh view in row-major order, its pixels spread over
    the map with a little jitter, so screen tiles cover compact texel boxes."""
    rng = np.random.default_rng(seed)
    x, y = np.meshgrid(np.arange(vw), np.arange(vh))
    u = (x.ravel() + rng.uniform(0.2, 0.8, vw * vh)) / vw * (1 + 2 * spill) - spill
    v = (y.ravel() + rng.uniform(0.2, 0.8, vw * vh)) / vh * (1 + 2 * spill) - spill
    z = rng.choice(np.array([0.4, 0.6, 0.8, 0.95], np.float32), vw * vh)
    return np.stack([u, v, z], 1).astype(np.float32)


def _long_edge_map():
    m = np.full((96, 96), 0.9, np.float32)
    m[10:70, 15:80] = 0.5
    m[75:90, 5:92] = 0.3
    m[20:60, 85:96] = 0.6
    m[0:4, :] = 0.7
    return m


@pytest.mark.parametrize("name", ["long_edges", "bars", "border", "checker2"])
def test_rpcf_long_traversals_leave_the_staged_band(rb, name):
    """Screen-ordered fragments (staged bands) over maps with long straight
    edges: traversals run past the steps staged beside the kernel's texels
    and go on in global memory, up to the map borders."""
    m = _long_edge_map() if name == "long_edges" else _adversarial_maps()[name]
    H, W = m.shape
    f = _screen_frags(W, H, 160, 120, seed=H + len(name))
    md, fd = dev(m), dev(f)
    for r, max_dist in ((2, 40), (5, 64), (3, 9), (1, 63), (11, 40)):
        say(f"rpcf long {name} r={r} maxd={max_dist}")
        p = dict(width=W, height=H, pitch=W, depth_bias=1e-4, max_dist=max_dist, kernel_radius=r, view_width=160)
        got = rb.rsmss_visibility(md, fd, p).cpu().numpy()
        check_soft(m, f, p, got, np.arange(0, len(f), 3))


def test_pitch_and_nonsquare_and_tiny_maps(rb):
    rng = np.random.default_rng(3)
    for (H, W, pitch) in [(1, 1, 1), (1, 7, 9), (5, 1, 4), (37, 53, 64), (200, 130, 131)]:
        full = np.zeros((H, pitch), np.float32)
        full[:, :W] = np.where(rng.random((H, W)) < 0.35, 0.5, 0.9)
        full[:, W:] = np.nan  # padding is never read
        m = np.ascontiguousarray(full[:, :W])
        f = _frags_for(W, H, 5000 + H, seed=H, spill=0.1)
        p = dict(width=W, height=H, pitch=pitch, depth_bias=1e-4, max_dist=8, kernel_radius=0)
        pd = dict(p, pitch=W)
        fd = dev(f)
        got_h = rb.rbsm_visibility(dev(full), fd, p).cpu().numpy()
        check_hard(m, f, pd, got_h)
        got_s = rb.rsmss_visibility(dev(full), fd, p).cpu().numpy()
        check_soft(m, f, pd, got_s)
        got_r = rb.rsmss_visibility(dev(full), fd, dict(p, kernel_radius=2)).cpu().numpy()
        check_soft(m, f, dict(pd, kernel_radius=2), got_r)


def test_nan_texels(rb):
    """A NaN texel compares false, so it is lit for every fragment (fragments
    themselves must be finite): both signs of NaN, every mode, staged and
    global reads (view_width 0 and 97)."""
    rng = np.random.default_rng(14)
    W = 48
    m = np.where(rng.random((W, W)) < 0.35, 0.5, 0.9).astype(np.float32)
    nan_p = np.float32(np.nan)
    nan_n = np.frombuffer(np.array([0xFFC00000], np.uint32).tobytes(), np.float32)[0]
    m[rng.random((W, W)) < 0.05] = nan_p
    m[rng.random((W, W)) < 0.05] = nan_n
    f = _frags_for(W, W, 6000, seed=14, spill=0.05)
    md, fd = dev(m), dev(f)
    for vw in (0, 97):
        p = dict(width=W, height=W, pitch=W, depth_bias=1e-4, max_dist=9, kernel_radius=0, view_width=vw)
        check_hard(m, f, p, rb.rbsm_visibility(md, fd, p).cpu().numpy())
        check_soft(m, f, p, rb.rsmss_visibility(md, fd, p).cpu().numpy())
        for r in (1, 3):
            pr = dict(p, kernel_radius=r)
            check_soft(m, f, pr, rb.rsmss_visibility(md, fd, pr).cpu().numpy())


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 257, 1000, 4099])
def test_ragged_sizes(rb, n):
    c = synth.make_config(1, 1005, small=True)
    f = np.ascontiguousarray(c["frags"][:n])
    got = rb.rbsm_visibility(dev(c["map"]), dev(f), c["params"]).cpu().numpy()
    check_hard(c["map"], f, c["params"], got)
    got = rb.rsmss_visibility(dev(c["map"]), dev(f), c["params"]).cpu().numpy()
    check_soft(c["map"], f, c["params"], got)


def test_empty_call(rb):
    c = synth.make_config(1, 1005, small=True)
    m = dev(c["map"])
    f = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    assert rb.rbsm_visibility(m, f, c["params"]).numel() == 0
    assert rb.rsmss_visibility(m, f, c["params"]).numel() == 0


def test_side_stream_ordering(rb):
    c = synth.make_config(2, 2002, small=True)
    s = torch.cuda.Stream()
    m, f = dev(c["map"]), dev(c["frags"])
    out = torch.full((len(c["frags"]),), 7, dtype=torch.uint8, device="cuda")
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        rb.rbsm_visibility(m, f, c["params"], out=out, stream=s)
        res = out.clone()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    check_hard(c["map"], c["frags"], c["params"], res.cpu().numpy())


def test_invalid_args_raise(rb):
    c = synth.make_config(1, 1005, small=True)
    m, f = dev(c["map"]), dev(c["frags"])
    with pytest.raises(rb.RbsmError):
        rb.rbsm_visibility(m, f, dict(c["params"], max_dist=0))
    with pytest.raises(rb.RbsmError):
        rb.rbsm_visibility(m, f, dict(c["params"], kernel_radius=3))
    with pytest.raises(rb.RbsmError):
        rb.rbsm_visibility(m, f.cpu(), c["params"])


def test_unaligned_pointers_take_the_scalar_path(rb):
    c = synth.make_config(2, 2003, small=True)
    n = len(c["frags"])
    buf = torch.zeros(3 * n + 8, dtype=torch.float32, device="cuda")
    fr = buf[1:1 + 3 * n]  # 4-byte aligned only
    fr.copy_(dev(c["frags"]).view(-1))
    m = dev(c["map"])
    ob = torch.zeros(n + 8, dtype=torch.uint8, device="cuda")
    got = rb.rbsm_visibility(m, fr, c["params"], out=ob[3:3 + n]).cpu().numpy()
    check_hard(c["map"], c["frags"], c["params"], got)
    of = torch.zeros(n + 8, dtype=torch.float32, device="cuda")
    got = rb.rsmss_visibility(m, fr, c["params"], out=of[1:1 + n]).cpu().numpy()
    check_soft(c["map"], c["frags"], c["params"], got)


def test_all_edge_fragments_fill_the_queue(rb):
    """Every fragment of every workgroup on an edge: the LDS queue runs full."""
    W = 64
    ii, jj = np.meshgrid(np.arange(W), np.arange(W))
    m = np.where((ii + jj) % 2 == 0, 0.5, 0.9).astype(np.float32)
    rng = np.random.default_rng(11)
    n = 3 * 1024 + 17
    f = np.stack([rng.uniform(0, 1, n), rng.uniform(0, 1, n), np.full(n, 0.9)], 1).astype(np.float32)
    for max_dist in (1, 7, 64):
        p = dict(width=W, height=W, pitch=W, depth_bias=1e-4, max_dist=max_dist, kernel_radius=0)
        check_hard(m, f, p, rb.rbsm_visibility(dev(m), dev(f), p).cpu().numpy())
        check_soft(m, f, p, rb.rsmss_visibility(dev(m), dev(f), p).cpu().numpy())


def test_largest_fragment_count(rb):
    """n = 2^31 - 1 fragments (the largest the boundary accepts: 25.8 GB of
    fragments, a ragged last tile), flat layout, hard, RSMSS and RPCF:
    sampled outputs, the last ones included, against the oracle."""
    c = synth.make_config(1, 1021, small=True)
    m = c["map"]
    n = 2 ** 31 - 1
    say(f"n = {n}: generating")
    g = torch.Generator(device="cuda").manual_seed(21)
    f = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    f[:, 0].uniform_(-0.02, 1.02, generator=g)
    f[:, 1].uniform_(-0.02, 1.02, generator=g)
    f[:, 2].uniform_(0.3, 0.95, generator=g)
    md = dev(m)
    p = dict(c["params"], view_width=0)
    rng = np.random.default_rng(22)
    idx = np.unique(np.concatenate([rng.integers(0, n, 3000), np.arange(n - 1100, n)]))
    ti = torch.from_numpy(idx).cuda()
    fs = f[ti].cpu().numpy()
    say("n = 2^31 - 1: hard")
    got = rb.rbsm_visibility(md, f, p)
    check_hard(m, fs, p, got[ti].cpu().numpy())
    del got
    say("n = 2^31 - 1: rsmss")
    got = rb.rsmss_visibility(md, f, p)
    check_soft(m, fs, p, got[ti].cpu().numpy())
    say("n = 2^31 - 1: rpcf r=1")
    pr = dict(p, kernel_radius=1)
    got = rb.rsmss_visibility(md, f, pr, out=got)
    check_soft(m, fs, pr, got[ti].cpu().numpy())
    del got, f
    torch.cuda.empty_cache()


def test_both_index_forms_at_their_boundary(rb):
    """A 4096-pixel-wide view (32 x 32 tiles) with the most fragments the
    32-bit index form takes (n + 32 * 4096 + 32 < 2^28: 3.2 GB of fragments,
    byte offsets up to 3.2e9) and one fragment more (the 64-bit form), hard
    and RSMSS: sampled outputs, the ragged last row included, against the
    oracle."""
    c = synth.make_config(1, 1023, small=True)
    m = c["map"]
    vw = 4096
    n32 = (1 << 28) - 32 * vw - 32 - 1
    say(f"index forms: generating {n32 + 1} fragments")
    g = torch.Generator(device="cuda").manual_seed(23)
    f = torch.empty((n32 + 1, 3), dtype=torch.float32, device="cuda")
    f[:, 0].uniform_(-0.02, 1.02, generator=g)
    f[:, 1].uniform_(-0.02, 1.02, generator=g)
    f[:, 2].uniform_(0.3, 0.95, generator=g)
    md = dev(m)
    p = dict(c["params"], view_width=vw)
    rng = np.random.default_rng(24)
    for n in (n32, n32 + 1):
        idx = np.unique(np.concatenate([rng.integers(0, n, 3000), np.arange(n - 5000, n),
                                        np.arange((1 << 27) - 600, (1 << 27) + 600)]))
        ti = torch.from_numpy(idx).cuda()
        fs = f[ti].cpu().numpy()
        fn = f[:n]
        say(f"index forms: n = {n} hard")
        got = rb.rbsm_visibility(md, fn, p)
        check_hard(m, fs, p, got[ti].cpu().numpy())
        del got
        say(f"index forms: n = {n} rsmss")
        got = rb.rsmss_visibility(md, fn, p)
        check_soft(m, fs, p, got[ti].cpu().numpy())
        del got
    del f
    torch.cuda.empty_cache()


@pytest.mark.parametrize("horizontal", [True, False])
def test_long_walks_overflow_the_continuation_queue(rb, horizontal):
    """Stripes one texel wide: every fragment is an edge fragment whose walks
    along the stripe run to the bound, so the walks still running after their
    first steps outnumber the continuation queue and the rest finish in place."""
    W = 64
    ii, jj = np.meshgrid(np.arange(W), np.arange(W))
    m = np.where((jj if horizontal else ii) % 2 == 0, 0.5, 0.9).astype(np.float32)
    rng = np.random.default_rng(12)
    n = 4 * 1024 + 5
    f = np.stack([rng.uniform(0, 1, n), rng.uniform(0, 1, n), np.full(n, 0.9)], 1).astype(np.float32)
    for max_dist in (3, 30, 64):
        p = dict(width=W, height=W, pitch=W, depth_bias=1e-4, max_dist=max_dist, kernel_radius=0)
        say(f"stripes horizontal={horizontal} max_dist={max_dist}")
        check_hard(m, f, p, rb.rbsm_visibility(dev(m), dev(f), p).cpu().numpy())
        check_soft(m, f, p, rb.rsmss_visibility(dev(m), dev(f), p).cpu().numpy())


def test_map_of_4_gib_takes_64_bit_walks(rb):
    """A 32768 x 32768 map (2^32 bytes): texel offsets no longer fit 32 bits,
    so walks step with 64-bit addresses.  Fragments sit on the edges of
    blockers in the last rows (offsets past 4 GiB) and the first ones."""
    S = 32768
    say("4 GiB map: building")
    m = np.full((S, S), 0.9, np.float32)
    rng = np.random.default_rng(13)
    rects = []
    for k in range(40):
        far = k % 2 == 0
        y0 = int(rng.integers(S - 300, S - 20)) if far else int(rng.integers(0, 280))
        x0 = int(rng.integers(0, S - 200))
        h, w = int(rng.integers(1, 40)), int(rng.integers(1, 60))
        m[y0:y0 + h, x0:x0 + w] = 0.5
        rects.append((x0, y0, w, h))
    # fragments on and next to the rectangles' borders
    fr = []
    for (x0, y0, w, h) in rects:
        xs = rng.uniform(x0 - 3, x0 + w + 3, 2000)
        ys = rng.uniform(y0 - 3, y0 + h + 3, 2000)
        fr.append(np.stack([xs / S, ys / S], 1))
    uv = np.concatenate(fr)
    f = np.concatenate([uv, np.full((len(uv), 1), 0.7)], 1).astype(np.float32)
    md = dev(m)
    fd = dev(f)
    for max_dist in (4, 40):
        p = dict(width=S, height=S, pitch=S, depth_bias=1e-4, max_dist=max_dist, kernel_radius=0)
        say(f"4 GiB map: max_dist={max_dist}")
        check_hard(m, f, p, rb.rbsm_visibility(md, fd, p).cpu().numpy())
        check_soft(m, f, p, rb.rsmss_visibility(md, fd, p).cpu().numpy())
        pr = dict(p, kernel_radius=2)
        check_soft(m, f, pr, rb.rsmss_visibility(md, fd, pr).cpu().numpy())
    del md
    torch.cuda.empty_cache()


@pytest.mark.parametrize("vw", [0, 1, 7, 240, 241, 1000])
def test_layout_hint_never_changes_results(rb, vw):
    """view_width only changes how fragments are tiled (2-D tiles, partial
    rows, flat chunks), never a result."""
    c = synth.make_config(2, 2004, small=True)
    f = np.ascontiguousarray(c["frags"][:30001])
    p = dict(c["params"], view_width=vw)
    md, fd = dev(c["map"]), dev(f)
    check_hard(c["map"], f, p, rb.rbsm_visibility(md, fd, p).cpu().numpy())
    check_soft(c["map"], f, p, rb.rsmss_visibility(md, fd, p).cpu().numpy())


def test_tiles_too_large_for_lds_read_global(rb):
    """Uniformly scattered fragments tiled 2-D: every tile's box exceeds the
    LDS capacity and the pass reads the map from global memory."""
    c = synth.make_config(1, 1009)
    p = dict(c["params"], view_width=256)
    md, fd = dev(c["map"]), dev(c["frags"])
    check_hard(c["map"], c["frags"], p, rb.rbsm_visibility(md, fd, p).cpu().numpy())
    check_soft(c["map"], c["frags"], p, rb.rsmss_visibility(md, fd, p).cpu().numpy())


@pytest.mark.parametrize("tw", [16, 32, 64])
@pytest.mark.parametrize("cap", [0, 256, 2048, 12288])  # 0: direct reads, nothing staged
def test_tuning_never_changes_results(rb, tw, cap):
    c = synth.make_config(2, 2006, small=True)
    md, fd = dev(c["map"]), dev(c["frags"])
    p = c["params"]
    want_h = rb.rbsm_visibility(md, fd, p).cpu().numpy()
    want_s = rb.rsmss_visibility(md, fd, p).cpu().numpy()
    for apron in (1, 4, 8):
        t = rb.RbsmTuning(tw, apron, cap)
        assert np.array_equal(rb.rbsm_pass_tuned(0, md, fd, p, t).cpu().numpy(), want_h)
        assert np.array_equal(rb.rbsm_pass_tuned(1, md, fd, p, t).cpu().numpy(), want_s)
    check_hard(c["map"], c["frags"], p, want_h)
