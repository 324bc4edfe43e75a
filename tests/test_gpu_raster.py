"""On-device shadow-map rasterization against the oracle's rasterizer.

Coverage is decided in binary64 on both sides and depths are binary32
minima, so maps must be bit-equal: whole maps at sizes the oracle finishes
quickly, sampled texels at full workload sizes, and the edge cases (tiny and
padded maps, no primitives, primitives the tile lists cannot hold, primitives
outside the map, malformed records, equal and NaN depths).  End to end, a
map rasterized on the device feeds the shadow pass to the same result as the
oracle's map.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import paper_1711_07793_amd as rb
    rb.load_library()
    return rb


def say(msg):
    print(msg, flush=True)


def dev_prims(prims):
    return torch.from_numpy(np.ascontiguousarray(prims).view(np.uint8).copy()).cuda()


def gpu_raster(rb, prims, rec, W, H):
    return rb.rbsm_rasterize(dev_prims(prims), rec, W, H).cpu().numpy()


@pytest.mark.parametrize("kind,W,H", [("quad", 512, 512), ("tris", 384, 256), ("fence", 512, 512),
                                      ("tris", 97, 131)])
def test_whole_maps_match_the_oracle(rb, kind, W, H):
    say(f"raster {kind} {W}x{H}")
    if kind == "quad":
        sc = synth.quad_scene(601, W, H)
    else:
        sc = synth.triangle_scene(602 + W, W, H, 128, fence=(kind == "fence"))
    prims, rec = sc.primitives()
    got = gpu_raster(rb, prims, rec, W, H)
    assert np.array_equal(got, oracle.raster(prims, rec, W, H))


@pytest.mark.parametrize("S,n_tris,fence", [(2048, 64, False), (4096, 256, True), (8192, 64, False)])
def test_full_size_maps_sampled(rb, S, n_tris, fence):
    say(f"raster full {S} tris={n_tris} fence={fence}")
    sc = synth.triangle_scene(700 + S, S, S, n_tris, fence=fence)
    prims, rec = sc.primitives()
    got = gpu_raster(rb, prims, rec, S, S)
    rng = np.random.default_rng(S)
    ti = rng.integers(0, S, 20000)
    tj = rng.integers(0, S, 20000)
    # also every texel of a few rows and columns, which cross primitive edges
    rows = rng.integers(0, S, 3)
    ti = np.concatenate([ti, np.tile(np.arange(S), 3)])
    tj = np.concatenate([tj, np.repeat(rows, S)])
    want = oracle.raster_texels(prims, rec, S, S, ti, tj)
    assert np.array_equal(got[tj, ti], want)


def test_padded_tiny_and_empty(rb):
    sc = synth.triangle_scene(611, 64, 64, 16, fence=True)
    prims, rec = sc.primitives()
    for (W, H) in [(1, 1), (3, 2), (33, 65), (64, 64)]:
        assert np.array_equal(gpu_raster(rb, prims, rec, W, H), oracle.raster(prims, rec, W, H)), (W, H)
    # no primitives: the receiver plane
    empty = np.zeros(0, oracle.PRIM_DTYPE)
    assert np.array_equal(gpu_raster(rb, empty, (0.9, 0.05, 0.03), 40, 30),
                          oracle.raster(empty, (0.9, 0.05, 0.03), 40, 30))
    # a pitched map: columns past the width are left alone
    out = torch.full((30, 48), -7.0, dtype=torch.float32, device="cuda")
    rb.rbsm_rasterize(dev_prims(prims), rec, 40, 30, out=out)
    o = out.cpu().numpy()
    assert np.array_equal(o[:, :40], oracle.raster(prims, rec, 40, 30))
    assert np.all(o[:, 40:] == -7.0)


@pytest.mark.parametrize("pitch,offset", [(45, 0), (48, 1), (64, 2), (44, 0)])
def test_row_alignment(rb, pitch, offset):
    """Rows that start 16-byte aligned take one 4-texel store per thread, the
    others texel by texel: both leave the same map and touch nothing past
    the width."""
    sc = synth.triangle_scene(612, 41, 37, 24, fence=True)
    prims, rec = sc.primitives()
    W, H = 41, 37
    buf = torch.full((H * pitch + offset + 8,), -7.0, dtype=torch.float32, device="cuda")
    out = buf[offset:offset + H * pitch].view(H, pitch)
    rb.rbsm_rasterize(dev_prims(prims), rec, W, H, out=out)
    o = out.cpu().numpy()
    assert np.array_equal(o[:, :W].view(np.uint32), oracle.raster(prims, rec, W, H).view(np.uint32))
    assert np.all(o[:, W:] == -7.0)
    b = buf.cpu().numpy()
    assert np.all(b[:offset] == -7.0) and np.all(b[offset + H * pitch:] == -7.0)


def test_thousands_of_overlapping_primitives(rb):
    """3000 large triangles over one 64^2 map: each tile sees all of them;
    those covering it whole fold into one depth, the rest are listed."""
    rng = np.random.default_rng(12)
    n = 3000
    p = np.zeros(n, oracle.PRIM_DTYPE)
    c = rng.uniform(0.2, 0.8, (n, 2))
    for k in range(n):
        ang = rng.uniform(0, 2 * np.pi, 3)
        ang.sort()
        r = rng.uniform(0.3, 0.6)
        p[k]["kind"], p[k]["nv"] = 0, 3
        p[k]["x"][:3] = c[k, 0] + r * np.cos(ang)   # counter-clockwise, large: all overlap every tile
        p[k]["y"][:3] = c[k, 1] + r * np.sin(ang)
        p[k]["depth"] = rng.uniform(0.1, 0.8)
    rec = (0.9, 0.0, 0.0)
    assert np.array_equal(gpu_raster(rb, p, rec, 64, 64), oracle.raster(p, rec, 64, 64))


def test_small_primitives_overflow_the_tile_list(rb):
    """3000 small triangles inside one 32 x 32 tile: they only partly cover
    it, so the tile lists more than its capacity and tests every primitive."""
    rng = np.random.default_rng(13)
    n = 3000
    p = np.zeros(n, oracle.PRIM_DTYPE)
    c = rng.uniform(0.05, 0.45, (n, 2))
    for k in range(n):
        ang = np.sort(rng.uniform(0, 2 * np.pi, 3))
        r = rng.uniform(0.005, 0.03)
        p[k]["kind"], p[k]["nv"] = 0, 3
        p[k]["x"][:3] = c[k, 0] + r * np.cos(ang)
        p[k]["y"][:3] = c[k, 1] + r * np.sin(ang)
        p[k]["depth"] = rng.uniform(0.1, 0.8)
    rec = (0.9, 0.0, 0.0)
    assert np.array_equal(gpu_raster(rb, p, rec, 64, 64), oracle.raster(p, rec, 64, 64))


def test_equal_depths_take_the_lowest_index(rb):
    """+0 and -0 compare equal: among equal depths the receiver plane wins,
    then the primitive of lowest index, in both orders; NaN depths never win.
    Bits are compared, so the sign of a zero counts."""
    def quad(x0, y0, x1, y1, z):
        q = np.zeros(1, oracle.PRIM_DTYPE)
        q["kind"], q["nv"] = 0, 4
        q["x"][0, :4] = [x0, x1, x1, x0]
        q["y"][0, :4] = [y0, y0, y1, y1]
        q["depth"] = z
        return q
    big = (-0.5, -0.5, 1.5, 1.5)
    cases = [
        np.concatenate([quad(*big, 0.0), quad(*big, -0.0)]),
        np.concatenate([quad(*big, -0.0), quad(*big, 0.0)]),
        np.concatenate([quad(0.1, 0.1, 0.7, 0.6, np.nan), quad(0.2, 0.3, 0.9, 0.8, 0.3),
                        quad(0.0, 0.0, 0.5, 0.5, 0.3), quad(*big, np.nan)]),
    ]
    for rec in ((0.9, 0.0, 0.0), (0.0, 0.0, 0.0), (-0.0, 0.0, 0.0)):
        for pr in cases:
            for (W, H) in ((64, 64), (45, 70)):
                got = gpu_raster(rb, pr, rec, W, H)
                want = oracle.raster(pr, rec, W, H)
                assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (rec, W, H, pr["depth"])


def test_outside_and_malformed_primitives(rb):
    p = np.zeros(5, oracle.PRIM_DTYPE)
    p[0]["kind"], p[0]["nv"] = 0, 3                      # entirely outside the map
    p[0]["x"][:3] = [1.5, 2.0, 1.7]
    p[0]["y"][:3] = [1.5, 1.6, 2.0]
    p[0]["depth"] = 0.2
    p[1]["kind"], p[1]["nv"] = 0, 7                      # bad vertex count: covers nothing
    p[1]["depth"] = 0.1
    p[2]["kind"] = 9                                     # unknown kind: covers nothing
    p[2]["depth"] = 0.1
    p[3]["kind"], p[3]["nv"] = 0, 4                      # quad overhanging the border
    p[3]["x"][:4] = [-0.3, 0.4, 0.4, -0.3]
    p[3]["y"][:4] = [-0.2, -0.2, 0.5, 0.5]
    p[3]["depth"] = 0.3
    p[4]["kind"], p[4]["nx"], p[4]["ny"] = 1, 0.6, 0.8   # slab
    p[4]["o"], p[4]["w"], p[4]["depth"] = 0.7, 0.05, 0.25
    rec = (0.9, 0.02, 0.01)
    assert np.array_equal(gpu_raster(rb, p, rec, 100, 80), oracle.raster(p, rec, 100, 80))


def test_device_map_feeds_the_pass(rb):
    """Rasterize on the device, shade on the device: the same masks as the
    oracle's raster shaded by the oracle."""
    c = synth.make_config(2, 2006, small=True)
    prims, rec = c["scene"].primitives()
    W = c["params"]["width"]
    m = rb.rbsm_rasterize(dev_prims(prims), rec, W, W)
    f = torch.from_numpy(c["frags"]).cuda()
    got = rb.rbsm_visibility(m, f, c["params"]).cpu().numpy()
    om = oracle.raster(prims, rec, W, W)
    assert np.array_equal(got, oracle.rbsm_hard(om, c["frags"], c["params"]))


def test_invalid_arguments(rb):
    p = dev_prims(np.zeros(2, oracle.PRIM_DTYPE))
    with pytest.raises(rb.RbsmError):
        rb.rbsm_rasterize(p, (0.9, 0, 0), 0, 10)
    with pytest.raises(rb.RbsmError):
        rb.rbsm_rasterize(p[:100], (0.9, 0, 0), 10, 10)   # not whole records
