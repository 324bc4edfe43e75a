"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check is a value printed in
the paper (Table 1, Fig. 3), a closed form (traversal lengths on strips), a
special case that reduces to a textbook routine (Williams' shadow test), an
independently structured implementation on exhaustive inputs (array stencils,
``stencil_rbsm.py``), a geometric ground truth (analytic half-planes), or an
exact symmetry of the method.
"""
import os

import numpy as np
import pytest

import oracle
import stencil_rbsm
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LIT, BLOCK = np.float32(0.9), np.float32(0.5)


def params(W, H=None, bias=0.0, max_dist=16, radius=0):
    H = W if H is None else H
    return dict(width=W, height=H, pitch=W, depth_bias=bias, max_dist=max_dist, kernel_radius=radius)


# --------------------------------------------------------------------------
# Table 1 / Eq. 4: compressed discontinuity for all 2^5 centre + neighbour patterns
# --------------------------------------------------------------------------

def _table1():
    rows = {}
    with open(os.path.join(GOLDEN, "table1_discontinuity.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            val, dx, dy, dz = [c.strip() for c in line.split("|")]
            rows[float(val)] = (dx, dy, dz)
    return rows


def test_table1_all_patterns():
    rows = _table1()
    dx_of = {v: m[0] for v, m in rows.items() if m[0] != "-"}
    dy_of = {v: m[1] for v, m in rows.items() if m[1] != "-"}
    dz_of = {v: m[2] for v, m in rows.items() if m[2] != "-"}
    # Eq. 4 weights the top (+y) neighbour by 2: the printed d.y labels for 0.25
    # and 0.5 are read swapped (the listing is authoritative).
    dy_read = {v: {"top": "bottom", "bottom": "top"}.get(m, m) for v, m in dy_of.items()}
    for centre_lit in (0, 1):
        for nb in range(16):
            m = np.full((5, 5), LIT, np.float32)
            c = LIT if centre_lit else BLOCK
            m[2, 2] = c
            other = BLOCK if centre_lit else LIT
            flags = [(nb >> k) & 1 for k in range(4)]  # left, right, top, bottom differ?
            for k, (di, dj) in enumerate([(-1, 0), (1, 0), (0, 1), (0, -1)]):
                m[2 + dj, 2 + di] = other if flags[k] else c
            frag = [(2.5) / 5, (2.5) / 5, 0.9]
            d = oracle.detail(m, frag, params(5), hard=False)
            left, right, top, bottom = flags
            want_x = {(0, 0): "none", (0, 1): "right", (1, 0): "left", (1, 1): "left-right"}[(left, right)]
            want_y = {(0, 0): "none", (1, 0): "top", (0, 1): "bottom", (1, 1): "top-bottom"}[(top, bottom)]
            want_z = "lit" if centre_lit else "shadowed"
            assert dx_of[float(d.d[0])] == want_x, (centre_lit, flags, list(d.d))
            assert dy_read[float(d.d[1])] == want_y, (centre_lit, flags, list(d.d))
            assert dz_of[float(d.d[2])] == want_z, (centre_lit, flags, list(d.d))
            # no discontinuity -> the plain test, no traversal (Listing 1)
            if nb == 0:
                assert d.path == 1 and d.vis == centre_lit


# --------------------------------------------------------------------------
# Fig. 3: the four shapes and the L-shape worked example
# --------------------------------------------------------------------------

def _fig3():
    shapes = {}
    with open(os.path.join(GOLDEN, "fig3_shapes.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, black, lit, expect = [c.strip() for c in line.split("|")]
            pts = lambda s: [tuple(int(v) for v in p.split(",")) for p in s.split()]
            shapes[name] = (pts(black), pts(lit), expect)
    return shapes


@pytest.mark.parametrize("bias", [0.0, 1e-4])
@pytest.mark.parametrize("shape", ["I", "U", "L", "O"])
def test_fig3_shapes(shape, bias):
    black, lit, expect = _fig3()[shape]
    W, off = 16, 6
    m = np.full((W, W), LIT, np.float32)
    for x, y in black:
        m[off + y, off + x] = BLOCK
    frags, xy = [], []
    for tx, ty in lit:
        for a in range(5):
            for b in range(5):
                x, y = tx + 0.1 + 0.2 * a, ty + 0.1 + 0.2 * b
                frags.append(((off + x) / W, (off + y) / W, 0.9))
                xy.append((x, y))
    frags = np.array(frags, np.float32)
    xy = np.array(xy)
    p = params(W, bias=bias)
    sm = oracle.shadow_map(m, frags, p)
    assert np.all(sm == 1), "the checked texels are the lit ones of the figure"
    hard = oracle.rbsm_hard(m, frags, p)
    if expect == "lit":
        assert np.all(hard == 1)
    elif expect == "shadowed":
        assert np.all(hard == 0)
    else:
        cols = [tuple(float(v) for v in c.split(",")) for c in expect.split()[1:]]
        want = np.zeros(len(xy), bool)
        for x0, x1, top in cols:
            want |= (xy[:, 0] >= x0) & (xy[:, 0] < x1) & (xy[:, 1] < top)
        assert np.array_equal(hard == 0, want)
        # the same set is the half-plane under the line from (2,3) to (3,1)
        below = (xy[:, 1] - 3.0) < -2.0 * (xy[:, 0] - 2.0)
        assert np.array_equal(hard == 0, below)
        assert int((hard == 0).sum()) == 25


# --------------------------------------------------------------------------
# Traversal lengths: closed form on strip patterns
# --------------------------------------------------------------------------

def _strip_case(n, stop, W=48, H=9):
    """Fragment texel (10, 4) lit with a shadowed texel below; the n texels to
    its right share that bottom discontinuity; then the strip stops by an
    opposite test ("end"), by a texel without the discontinuity ("leave"), or
    by the map border ("border")."""
    x0, y0 = 10, 4
    if stop == "border":
        W = x0 + n + 1
    m = np.full((H, W), LIT, np.float32)
    for x in range(x0, x0 + n + 1):
        m[y0 - 1, x] = BLOCK
    if stop == "end":
        m[y0, x0 + n + 1] = BLOCK
    frag = np.array([(x0 + 0.375) / W, (y0 + 0.625) / H, 0.9], np.float32)
    return m, frag


def _transform(m, frag, how):
    """Map + fragment mirrored in x ("mirror"), transposed ("transpose") or both."""
    u, v, z = [float(t) for t in frag]
    H, W = m.shape
    if how in ("mirror", "transpose_mirror"):
        m = m[:, ::-1]
        u = 1.0 - u
    if how in ("transpose", "transpose_mirror"):
        m = m.T
        u, v = v, u
    return np.ascontiguousarray(m), np.array([u, v, z], np.float32)


@pytest.mark.parametrize("max_dist", [1, 2, 3, 16])
@pytest.mark.parametrize("stop", ["end", "leave", "border"])
def test_traversal_closed_form(max_dist, stop):
    # walk index in rd (left, right, top, bottom) after each transform of a
    # construction that walks to the right
    walk_index = {"none": 1, "mirror": 0, "transpose": 2, "transpose_mirror": 3}
    for n in range(0, max_dist + 3):
        m0, f0 = _strip_case(n, stop)
        D = min(n + 1, max_dist + 1)
        want = D if (stop == "end" and n + 1 <= max_dist) else -D
        if stop == "border":  # clamp-to-edge repeats the last strip texel: the walk runs out
            want = -(max_dist + 1)
        for how, idx in walk_index.items():
            m, f = (m0, f0) if how == "none" else _transform(m0, f0, how)
            H, W = m.shape
            d = oracle.detail(m, f, params(W, H, max_dist=max_dist), hard=True)
            assert d.path == 2
            assert d.rd[idx] == want, (n, stop, how, list(d.rd))
            # the walk opposite the strip leaves the edge at once
            opp = {0: 1, 1: 0, 2: 3, 3: 2}[idx]
            assert d.rd[opp] == -1, (n, stop, how, list(d.rd))


# --------------------------------------------------------------------------
# Exhaustive 4x4 binary maps against the array-stencil implementation
# --------------------------------------------------------------------------

def _all_4x4():
    idx = np.arange(1 << 16)
    bits = (idx[:, None] >> np.arange(16)[None, :]) & 1  # bit b -> texel (b % 4, b // 4)
    blocked = bits.reshape(-1, 4, 4).astype(bool)
    return blocked


@pytest.mark.parametrize("hard", [True, False])
@pytest.mark.parametrize("max_dist", [1, 2, 3, 16])
def test_exhaustive_4x4_against_stencil(max_dist, hard):
    blocked = _all_4x4()
    n_maps = blocked.shape[0]
    maps = np.where(blocked, BLOCK, LIT).astype(np.float32)
    S = (~blocked).astype(np.uint8)
    mi = np.repeat(np.arange(n_maps, dtype=np.int32), 16)
    t = np.tile(np.arange(16), n_maps)
    ti, tj = t % 4, t // 4
    kx = (mi.astype(np.int64) * 5 + t * 3 + max_dist) % 64
    ky = (mi.astype(np.int64) * 11 + t * 7 + 3 * max_dist) % 64
    fx = ((2 * kx + 1) / 128.0).astype(np.float32)
    fy = ((2 * ky + 1) / 128.0).astype(np.float32)
    frags = np.stack([(ti + fx) / 4.0, (tj + fy) / 4.0, np.full(ti.shape, 0.9)], 1).astype(np.float32)
    p = params(4, max_dist=max_dist)
    vis_o, rd_o, nrd_o = oracle.multi(maps, mi, frags, p, hard)
    chunk = 1 << 14
    for c0 in range(0, n_maps, chunk):
        sel = slice(c0 * 16, (c0 + chunk) * 16)
        vis_s, rd_s, nrd_s = stencil_rbsm.evaluate(S[c0:c0 + chunk], mi[sel] - c0, ti[sel], tj[sel],
                                                   fx[sel], fy[sel], max_dist, hard)
        assert np.array_equal(rd_o[sel], rd_s)
        assert np.array_equal(nrd_o[sel], nrd_s)
        assert np.array_equal(vis_o[sel], vis_s)
    # every discontinuity pattern and every walk length up to the bound occurs
    edge = np.any(rd_o != 0, axis=1)
    lengths = np.unique(np.abs(rd_o[edge]))
    assert lengths.min() == 1 and lengths.max() == min(max_dist + 1, 4 + max_dist)
    assert set(np.unique(rd_o[edge] > 0)) == {False, True}


def _blob_maps(seed, n, H, W):
    """Binary maps made of random overlapping rectangles: long runs, concave
    corners, lines one texel thick and shapes touching the border."""
    rng = np.random.default_rng(seed)
    blocked = np.zeros((n, H, W), bool)
    for k in range(n):
        for _ in range(int(rng.integers(2, 12))):
            x0, y0 = int(rng.integers(-4, W)), int(rng.integers(-4, H))
            w = int(rng.integers(1, W // 2)) if rng.random() < 0.8 else 1
            h = int(rng.integers(1, H // 2)) if rng.random() < 0.8 else 1
            blocked[k, max(y0, 0):max(y0 + h, 0), max(x0, 0):max(x0 + w, 0)] ^= True
    return blocked


@pytest.mark.parametrize("max_dist,hard", [(3, True), (16, True), (40, True), (3, False), (40, False)])
def test_random_blob_maps_against_stencil(max_dist, hard):
    """Non-square odd-sized maps whose runs exceed the walk bound: the oracle
    and the stencil form agree on every texel, walk and visibility."""
    H, W, n_maps = 37, 45, 24
    blocked = _blob_maps(1000 + max_dist + hard, n_maps, H, W)
    maps = np.where(blocked, BLOCK, LIT).astype(np.float32)
    S = (~blocked).astype(np.uint8)
    rng = np.random.default_rng(2000 + max_dist)
    mi = np.repeat(np.arange(n_maps, dtype=np.int32), H * W)
    t = np.tile(np.arange(H * W), n_maps)
    ti, tj = t % W, t // W
    u = ((ti + rng.uniform(0, 1, ti.shape)) / W).astype(np.float32)
    v = ((tj + rng.uniform(0, 1, tj.shape)) / H).astype(np.float32)
    # the texel and fraction the oracle derives from (u, v) in binary32
    X, Y = u * np.float32(W), v * np.float32(H)
    ti, tj = np.floor(X).astype(np.int64), np.floor(Y).astype(np.int64)
    ok = (ti < W) & (tj < H)
    mi, ti, tj, u, v, X, Y = mi[ok], ti[ok], tj[ok], u[ok], v[ok], X[ok], Y[ok]
    fx, fy = (X - np.floor(X)).astype(np.float32), (Y - np.floor(Y)).astype(np.float32)
    frags = np.stack([u, v, np.full(u.shape, 0.9, np.float32)], 1).astype(np.float32)
    vis_o, rd_o, nrd_o = oracle.multi(maps, mi, frags, params(W, H, max_dist=max_dist), hard)
    vis_s, rd_s, nrd_s = stencil_rbsm.evaluate(S, mi, ti, tj, fx, fy, max_dist, hard)
    assert np.array_equal(rd_o, rd_s)
    assert np.array_equal(nrd_o, nrd_s)
    assert np.array_equal(vis_o, vis_s)
    # walks of every kind occur: ends, leaves and bound-exhausted ones
    assert (rd_o > 0).any() and (rd_o < 0).any()
    assert (rd_o == -(max_dist + 1)).any() == (max_dist < max(H, W))


# --------------------------------------------------------------------------
# Check (a): plain shadow mapping wherever no discontinuity exists
# --------------------------------------------------------------------------

def _textbook_tests(map_, frags, p):
    """Williams' shadow test at the fragment's texel and its 4 neighbours (clamped)."""
    W, H = p["width"], p["height"]
    X = frags[:, 0] * np.float32(W)
    Y = frags[:, 1] * np.float32(H)
    i0 = np.floor(X).astype(np.int64)
    j0 = np.floor(Y).astype(np.int64)
    zb = (frags[:, 2] - np.float32(p["depth_bias"])).astype(np.float32)

    def lit(di, dj):
        i = np.clip(i0 + di, 0, W - 1)
        j = np.clip(j0 + dj, 0, H - 1)
        return ~(zb > map_[j, i])

    return lit(0, 0), [lit(-1, 0), lit(1, 0), lit(0, 1), lit(0, -1)]


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_plain_sm_where_no_discontinuity(cfg):
    c = synth.make_config(cfg, 1000 * cfg + 1, small=True)
    m, f, p = c["map"], c["frags"], c["params"]
    centre, nb = _textbook_tests(m, f, p)
    flat = np.all([n == centre for n in nb], axis=0)
    assert flat.mean() > 0.5
    sm = oracle.shadow_map(m, f, p)
    assert np.array_equal(sm.astype(bool), centre)
    hard = oracle.rbsm_hard(m, f, p)
    soft = oracle.rsmss(m, f, p)
    assert np.array_equal(hard[flat], sm[flat])
    assert np.array_equal(soft[flat], sm[flat].astype(np.float32))
    # hard recovery works on the lit side only: shadowed stays shadowed
    assert np.all(hard[sm == 0] == 0)
    assert np.all((soft >= 0) & (soft <= 1))
    assert (~flat).sum() > 0


# --------------------------------------------------------------------------
# Check (c): analytic half-plane blockers at random angles
# --------------------------------------------------------------------------

def _halfplane(theta, off, W=64, S=8, conservative=False):
    n = np.array([np.cos(theta), np.sin(theta)])
    c = n @ np.array([W / 2, W / 2]) + off
    ii, jj = np.meshgrid(np.arange(W), np.arange(W))
    if conservative:  # a texel blocks only if the half-plane covers all of it
        inside = np.ones(ii.shape, bool)
        for dx in (0, 1):
            for dy in (0, 1):
                inside &= n[0] * (ii + dx) + n[1] * (jj + dy) < c
    else:  # centre sampling
        inside = n[0] * (ii + 0.5) + n[1] * (jj + 0.5) < c
    m = np.where(inside, BLOCK, LIT).astype(np.float32)
    g = (np.arange(W * S) + 0.5) / S
    X, Y = np.meshgrid(g, g)
    fr = np.stack([X.ravel() / W, Y.ravel() / W, np.full(X.size, 0.9)], 1).astype(np.float32)
    truth = (n[0] * X + n[1] * Y < c)
    p = params(W, bias=1e-4, max_dist=16)
    sm = (oracle.shadow_map(m, fr, p) == 0).reshape(X.shape)
    hard = (oracle.rbsm_hard(m, fr, p) == 0).reshape(X.shape)
    soft = oracle.rsmss(m, fr, p).reshape(X.shape)
    inner = (X > 8) & (X < W - 8) & (Y > 8) & (Y < W - 8)
    return truth, sm, hard, soft, inner


def test_halfplane_filtered_closer_than_sm():
    rng = np.random.default_rng(1711)
    miss_sm = miss_soft = 0
    for _ in range(24):
        truth, sm, hard, soft, inner = _halfplane(rng.uniform(0, 2 * np.pi), rng.uniform(-3, 3))
        miss_sm += int((sm != truth)[inner].sum())
        miss_soft += int(((soft < 0.5) != truth)[inner].sum())
    assert miss_soft < 0.6 * miss_sm, (miss_soft, miss_sm)


def test_halfplane_hard_closer_than_sm_on_conservative_maps():
    rng = np.random.default_rng(7793)
    miss_sm = miss_hard = 0
    for _ in range(24):
        truth, sm, hard, soft, inner = _halfplane(rng.uniform(0, 2 * np.pi), rng.uniform(-3, 3),
                                                  conservative=True)
        miss_sm += int((sm != truth)[inner].sum())
        miss_hard += int((hard != truth)[inner].sum())
    assert miss_hard < 0.6 * miss_sm, (miss_hard, miss_sm)


def test_halfplane_hard_edges_less_jagged_than_sm():
    """Std of the per-column boundary residual about the analytic edge
    (shallow edges, centre-sampled maps).  The hard mask is biased about half a
    texel toward shadow (the paper's shadow overestimation); the bias is
    reported, the jaggedness is gated."""
    rng = np.random.default_rng(31)
    W, S = 64, 8
    for _ in range(16):
        theta = np.pi / 2 + rng.uniform(-0.45, 0.45) + (np.pi if rng.random() < 0.5 else 0.0)
        truth, sm, hard, soft, inner = _halfplane(theta, rng.uniform(-3, 3), W, S)
        cols, band = slice(12 * S, (W - 12) * S), slice(4 * S, (W - 4) * S)
        ht = truth[band, cols].sum(0) / S
        r_sm = sm[band, cols].sum(0) / S - ht
        r_hard = hard[band, cols].sum(0) / S - ht
        r_soft = (soft < 0.5)[band, cols].sum(0) / S - ht
        assert r_hard.std() < 0.6 * r_sm.std(), (r_hard.std(), r_sm.std())
        assert r_soft.std() < 0.6 * r_sm.std(), (r_soft.std(), r_sm.std())
        assert 0.2 < r_hard.mean() < 0.8  # outward bias of about half a texel
        assert abs(r_soft.mean()) < 0.2


# --------------------------------------------------------------------------
# Symmetries ("symmetry-aware", Sec. 4)
# --------------------------------------------------------------------------

def _random_scene(seed, W=64, n_rect=14):
    rng = np.random.default_rng(seed)
    m = np.full((W, W), LIT, np.float32)
    for _ in range(n_rect):
        x0, y0 = rng.integers(0, W, 2)
        w, h = rng.integers(1, 18, 2)
        m[y0:y0 + h, x0:x0 + w] = np.float32(rng.choice([0.3, 0.5, 0.7]))
    n = 20000
    i = rng.integers(0, W, n)
    j = rng.integers(0, W, n)
    fx = (2 * rng.integers(0, 64, n) + 1) / 128.0
    fy = (2 * rng.integers(0, 64, n) + 1) / 128.0
    z = rng.choice(np.array([0.4, 0.6, 0.9], np.float32), n)
    fr = np.stack([(i + fx) / W, (j + fy) / W, z], 1).astype(np.float32)
    return m, fr


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mirror_symmetry_exact(seed):
    m, fr = _random_scene(seed)
    p = params(64, bias=1e-4, max_dist=16)
    h0, s0 = oracle.rbsm_hard(m, fr, p), oracle.rsmss(m, fr, p)
    mx = np.ascontiguousarray(m[:, ::-1])
    fx = fr.copy(); fx[:, 0] = np.float32(1.0) - fr[:, 0]
    my = np.ascontiguousarray(m[::-1, :])
    fy = fr.copy(); fy[:, 1] = np.float32(1.0) - fr[:, 1]
    for mm, ff in ((mx, fx), (my, fy)):
        assert np.array_equal(oracle.rbsm_hard(mm, ff, p), h0)
        assert np.array_equal(oracle.rsmss(mm, ff, p), s0)


@pytest.mark.parametrize("seed", [4, 5])
def test_transpose_symmetry(seed):
    m, fr = _random_scene(seed)
    p = params(64, bias=1e-4, max_dist=16)
    h0, s0 = oracle.rbsm_hard(m, fr, p), oracle.rsmss(m, fr, p)
    mt = np.ascontiguousarray(m.T)
    ft = fr[:, [1, 0, 2]].copy()
    h1, s1 = oracle.rbsm_hard(mt, ft, p), oracle.rsmss(mt, ft, p)
    diff = np.nonzero(h0 != h1)[0]
    for k in diff:  # only where the L line ties within rounding
        assert oracle.margin(m, fr[k], p, True) < 1e-6
    assert np.max(np.abs(s0 - s1)) <= 2.0 ** -22


# --------------------------------------------------------------------------
# RSMSS properties (Listing 5)
# --------------------------------------------------------------------------

def test_rsmss_shapes_and_consistency_with_hard():
    m, fr = _random_scene(9)
    p = params(64, bias=1e-4, max_dist=16)
    s = oracle.rsmss(m, fr, p)
    h = oracle.rbsm_hard(m, fr, p)
    assert np.all((s >= 0) & (s <= 1))
    n_checked = 0
    for k in range(0, fr.shape[0], 7):
        ds = oracle.detail(m, fr[k], p, hard=False)
        if ds.path != 2:
            continue
        d, nrd = list(ds.d), list(ds.nrd)
        cx, cy = nrd[2], nrd[3]
        if d[0] == 0.75 and d[1] == 0.75:      # short O flips the test
            assert ds.vis == d[2]
        elif cx == 1 and cy == 1:              # long O flips the test
            assert ds.vis == d[2]
        elif cx == 1:                          # U: linear in the other axis
            sg = 1 - 2 * d[2]
            assert ds.vis == np.float32(d[2] + sg * nrd[1])
        if d[2] == 0 and cx == 0 and cy == 0:  # lit L: hard == (RSMSS == 1)
            n_checked += 1
            if (s[k] == 1) != (h[k] == 1):
                assert oracle.margin(m, fr[k], p, True) < 1e-6
    assert n_checked > 20


# --------------------------------------------------------------------------
# RPCF: box average of RSMSS over texel offsets
# --------------------------------------------------------------------------

def test_rpcf_radius_zero_is_rsmss_and_constant_field_identity():
    m, fr = _random_scene(12)
    p0 = params(64, bias=1e-4, max_dist=16)
    s0 = oracle.rsmss(m, fr, p0)
    assert np.array_equal(oracle.rsmss(m, fr, dict(p0, kernel_radius=0)), s0)
    flat = np.full((64, 64), LIT, np.float32)
    for r in (1, 3):
        out = oracle.rsmss(flat, fr[:500], dict(p0, kernel_radius=r))
        assert np.all(out == 1.0)


def test_rpcf_matches_shifted_fragments_brute_force():
    m, fr = _random_scene(13, W=32, n_rect=6)
    fr = fr[:300].copy()
    fr[:, 0] = (np.floor(fr[:, 0] * 64) + 0.5) / 64  # keep in range after the W change
    fr[:, 1] = (np.floor(fr[:, 1] * 64) + 0.5) / 64
    m = np.ascontiguousarray(m[:32, :32])
    r = 2
    p = params(32, bias=1e-4, max_dist=16, radius=r)
    got = oracle.rsmss(m, fr, p)
    p0 = dict(p, kernel_radius=0)
    acc = np.zeros(fr.shape[0], np.float64)
    for a in range(-r, r + 1):
        for b in range(-r, r + 1):
            sh = fr.copy()
            sh[:, 0] = fr[:, 0] + np.float32(a / 32)
            sh[:, 1] = fr[:, 1] + np.float32(b / 32)
            acc += oracle.rsmss(m, sh, p0).astype(np.float64)
    want = (acc / 25.0).astype(np.float32)
    assert np.array_equal(got, want)
    assert np.any((got > 0) & (got < 1))  # the scene puts edges inside the boxes


# --------------------------------------------------------------------------
# Input validation and read instrumentation
# --------------------------------------------------------------------------

def test_oracle_rejects_bad_input():
    m = np.full((4, 4), LIT, np.float32)
    f = np.array([[0.5, 0.5, 0.9]], np.float32)
    with pytest.raises(ValueError):
        oracle.rbsm_hard(m, f, params(4, radius=1))
    with pytest.raises(ValueError):
        oracle.rbsm_hard(m, f, dict(params(4), pitch=2))
    with pytest.raises(ValueError):
        oracle.rsmss(m, np.array([[np.nan, 0.5, 0.9]], np.float32), params(4))


def test_read_counts():
    m = np.full((8, 8), LIT, np.float32)
    m[0, 0] = BLOCK
    p = params(8)
    # flat lit fragment: centre + 4 neighbours
    touch, reads = oracle.touched_texels(m, np.array([[0.55, 0.55, 0.9]], np.float32), p, hard=True)
    assert reads == 5 and touch.sum() == 5
    # shadowed fragment in hard mode: only the centre
    touch, reads = oracle.touched_texels(m, np.array([[0.05, 0.05, 0.9]], np.float32), p, hard=True)
    assert reads == 1 and touch.sum() == 1


# --------------------------------------------------------------------------
# Multi-light compositing (serving extension)
# --------------------------------------------------------------------------

def test_composite_worked_examples():
    rows = [list(map(float, ln.split())) for ln in open(os.path.join(GOLDEN, "composite_examples.txt"))
            if ln.strip() and not ln.startswith("#")]
    for r in rows:
        m = np.array([int(r[0])], np.uint8)
        a, b = np.array([r[1]], np.float32), np.array([r[2]], np.float32)
        got = oracle.composite([m, a, b], r[3:6])
        assert got[0] == np.float32(r[6]), r


def test_composite_identities():
    rng = np.random.default_rng(21)
    v = rng.random(1000).astype(np.float32)
    h = (rng.random(1000) < 0.5).astype(np.uint8)
    assert np.array_equal(oracle.composite([v], [1.0]), v)          # one light, weight 1
    assert np.array_equal(oracle.composite([h], [1.0]), h.astype(np.float32))
    assert np.array_equal(oracle.composite([v, h], [0.0, 0.0]), np.zeros(1000, np.float32))
    # power-of-two weights scale exactly; order of lights matters only through rounding
    assert np.array_equal(oracle.composite([v], [0.25]), v * np.float32(0.25))
    both = oracle.composite([v, h], [0.5, 0.5])
    assert np.max(np.abs(both.astype(np.float64) - 0.5 * (v + h))) <= 2 ** -24


# --------------------------------------------------------------------------
# Shadow-map rasterization (on-device extension)
# --------------------------------------------------------------------------

def _poly(xs, ys, depth):
    r = np.zeros(1, oracle.PRIM_DTYPE)
    r["kind"], r["nv"], r["depth"] = 0, len(xs), depth
    r["x"][0, :len(xs)] = xs
    r["y"][0, :len(ys)] = ys
    return r


def _slab(nx, ny, o, w, depth):
    r = np.zeros(1, oracle.PRIM_DTYPE)
    r["kind"], r["nx"], r["ny"], r["o"], r["w"], r["depth"] = 1, nx, ny, o, w, depth
    return r


def _exact_cover(prim, W, H):
    """Coverage of texel centres in exact rational arithmetic (vertices on a
    dyadic grid, so binary64 computes the same predicates exactly)."""
    from fractions import Fraction as F
    cov = np.zeros((H, W), bool)
    xs = [F(float(v)) for v in prim["x"][:prim["nv"]]]
    ys = [F(float(v)) for v in prim["y"][:prim["nv"]]]
    for j in range(H):
        py = F(2 * j + 1, 2 * H)
        for i in range(W):
            px = F(2 * i + 1, 2 * W)
            inside = True
            for a in range(prim["nv"]):
                b = (a + 1) % prim["nv"]
                c = (xs[b] - xs[a]) * (py - ys[a]) - (ys[b] - ys[a]) * (px - xs[a])
                if c < 0 or (c == 0 and not (ys[b] - ys[a] < 0 or (ys[b] == ys[a] and xs[b] - xs[a] < 0))):
                    inside = False
                    break
            cov[j, i] = inside
    return cov


def test_raster_receiver_plane_closed_form():
    W, H = 37, 23
    got = oracle.raster(np.zeros(0, oracle.PRIM_DTYPE), (0.9, 0.05, -0.03), W, H)
    u = (np.arange(W) + 0.5) / W
    v = (np.arange(H) + 0.5) / H
    want = (0.9 + 0.05 * (u[None, :] - 0.5) + -0.03 * (v[:, None] - 0.5)).astype(np.float32)
    assert np.array_equal(got, want)


def test_raster_matches_exact_rational_coverage():
    rng = np.random.default_rng(31)
    W = H = 32
    for _ in range(40):
        pts = rng.integers(0, 1025, size=(3, 2)) / 1024.0   # dyadic vertices, exact in binary64
        a = (pts[1, 0] - pts[0, 0]) * (pts[2, 1] - pts[0, 1]) - (pts[1, 1] - pts[0, 1]) * (pts[2, 0] - pts[0, 0])
        if a == 0:
            continue
        if a < 0:
            pts = pts[::-1]
        prim = _poly(pts[:, 0], pts[:, 1], 0.5)
        got = oracle.raster(prim, (0.9, 0.0, 0.0), W, H) == np.float32(0.5)
        assert np.array_equal(got, _exact_cover(prim[0], W, H))


def test_raster_shared_edges_are_watertight():
    """A square cut along a diagonal: every centre inside the square is
    covered by exactly one of the two halves, including centres on the cut."""
    W = H = 64
    # corners on texel centres, so centres (k + .5)/64 lie exactly on the cut
    x0 = y0 = 8.5 / 64
    x1 = y1 = 40.5 / 64
    lower = _poly([x0, x1, x1], [y0, y0, y1], 0.3)           # CCW
    upper = _poly([x0, x1, x0], [y0, y1, y1], 0.4)           # CCW
    both = np.concatenate([lower, upper])
    cl = oracle.raster(lower, (0.9, 0, 0), W, H) < 0.9
    cu = oracle.raster(upper, (0.9, 0, 0), W, H) < 0.9
    assert not np.any(cl & cu)
    square = _poly([x0, x1, x1, x0], [y0, y0, y1, y1], 0.3)
    cs = oracle.raster(square, (0.9, 0, 0), W, H) < 0.9
    assert np.array_equal(cl | cu, cs)
    assert np.any(np.diag(cl | cu))                          # centres on the cut are covered
    # the nearer primitive wins where both could apply
    m = oracle.raster(both, (0.9, 0, 0), W, H)
    assert set(np.unique(m).tolist()) <= {np.float32(0.3), np.float32(0.4), np.float32(0.9)}


def test_raster_slabs_cover_the_half_open_band():
    W = H = 64
    # vertical band 16/64 <= u < 24/64: texel columns 16..23 (their centres)
    s = _slab(1.0, 0.0, 16 / 64, 8 / 64, 0.2)
    cov = oracle.raster(s, (0.9, 0, 0), W, H) < 0.9
    assert np.array_equal(np.nonzero(cov.any(axis=0))[0], np.arange(16, 24))
    assert cov[:, 16:24].all()


@pytest.mark.parametrize("fence", [False, True])
def test_raster_agrees_with_the_scene_generator(fence):
    sc = synth.triangle_scene(77 + fence, 200, 150, 24, fence=fence)
    prims, rec = sc.primitives()
    assert np.array_equal(oracle.raster(prims, rec, 200, 150), sc.raster())
    q = synth.quad_scene(78, 128, 128)
    prims, rec = q.primitives()
    assert np.array_equal(oracle.raster(prims, rec, 128, 128), q.raster())


# --------------------------------------------------------------------------
# The binary64 decision margin (used to excuse hard-mask disagreements):
# pinned by hand-placed near-boundary texels and by the closed form of the
# revectorized edge in Fig. 3c
# --------------------------------------------------------------------------

FAR_LIT, FAR_BLOCK = np.float32(1.0), np.float32(0.25)


def _straight_edge(W=64, j0=20):
    """Rows below j0 blocked (0.25), the rest lit (1.0): a fragment at depth
    0.75 in row j0 sits on an edge whose left and right walks run the full
    MAXDIST (every visited texel shares the bottom discontinuity)."""
    m = np.full((W, W), FAR_LIT, np.float32)
    m[:j0, :] = FAR_BLOCK
    return m


@pytest.mark.parametrize("bias", [0.0, 2.0 ** -10])
@pytest.mark.parametrize("hard", [True, False])
def test_margin_single_near_boundary_texel(bias, hard):
    W, i0, j0, md = 64, 20, 20, 16
    z = np.float32(0.75 + bias)           # z - bias = 0.75 exactly
    p = params(W, bias=bias, max_dist=md)
    frag = np.array([(i0 + 0.375) / W, (j0 + 0.625) / W, z], np.float32)
    base = oracle.margin(_straight_edge(W, j0), frag, p, hard)
    assert base == 0.25                    # the lit texels 1.0 against 0.75
    d = oracle.detail(_straight_edge(W, j0), frag, p, hard)
    assert d.path == 2 and d.rd[0] == -(md + 1) and d.rd[1] == -(md + 1)
    for delta in (2.0 ** -10, 2.0 ** -20):
        placed = {
            "centre": (i0, j0, 0.75 + delta),
            "walk step MAXDIST": (i0 + md, j0, 0.75 + delta),
            "walk step -MAXDIST": (i0 - md, j0, 0.75 + delta),
            "side neighbour of a step": (i0 + 5, j0 - 1, 0.75 - delta),
            "vertical walk, its side neighbour": (i0 + 1, j0 + 3, 0.75 + delta),
        }
        for what, (i, j, t) in placed.items():
            m = _straight_edge(W, j0)
            m[j, i] = np.float32(t)
            # the placed texel keeps its test, so the walks are unchanged
            dd = oracle.detail(m, frag, p, hard)
            assert list(dd.rd) == list(d.rd), what
            assert oracle.margin(m, frag, p, hard) == delta, what
        for what, (i, j) in {"off the walk cross": (i0 + 2, j0 + 2),
                             "beyond the reach": (i0 + md + 2, j0)}.items():
            m = _straight_edge(W, j0)
            m[j, i] = np.float32(0.75 + delta)
            assert oracle.margin(m, frag, p, hard) == base, what


def test_margin_revectorized_edge_closed_form():
    """Fig. 3c: on the L window the edge line runs from (2,3) to (3,1); a lit
    fragment at (x, y) in texel (2,1) or (2,2) has nrd.x = x - 2 and
    nrd.y = (y - 1) / 2 (one end to the left, an edge two texels tall), so the
    decision value is |(y - 1)/2 - (1 - (x - 2))|, capped by the depth margin."""
    black, lit, _ = _fig3()["L"]
    W, off = 16, 6
    m = np.full((W, W), FAR_LIT, np.float32)
    for x, y in black:
        m[off + y, off + x] = np.float32(0.5)
    p = params(W)
    z = np.float32(0.875)  # depth margins 0.125 (lit) and 0.375 (blocked)
    n_line = 0
    for tx, ty in lit:
        for a in range(16):
            for b in range(16):
                x, y = tx + (2 * a + 1) / 32.0, ty + (2 * b + 1) / 32.0
                frag = np.array([(off + x) / W, (off + y) / W, z], np.float32)
                line = abs((y - 1.0) / 2.0 - (1.0 - (x - 2.0)))
                want = min(0.125, line)
                assert oracle.margin(m, frag, p, True) == want, (x, y)
                n_line += line < 0.125
    assert n_line > 100


# --------------------------------------------------------------------------
# RSMSS continuity across straight edges (Sec. 3.2: the origin of the
# normalized space stays at the edge, so the fake penumbra joins up at the
# side between a lit and a shadowed texel)
# --------------------------------------------------------------------------

def test_rsmss_continuous_across_straight_edges():
    rng = np.random.default_rng(3211)
    W, md, eps = 64, 16, 2.0 ** -12
    p = params(W, bias=1e-4, max_dist=md)
    lo, hi = md + 2, W - md - 2
    checked = 0
    for _ in range(10):
        while True:  # edges away from the axes: runs shorter than MAXDIST
            theta = rng.uniform(0, 2 * np.pi)
            if min(abs(np.sin(theta)), abs(np.cos(theta))) > 0.15:
                break
        n = np.array([np.cos(theta), np.sin(theta)])
        c = n @ np.array([W / 2, W / 2]) + rng.uniform(-2, 2)
        ii, jj = np.meshgrid(np.arange(W), np.arange(W))
        inside = n[0] * (ii + 0.5) + n[1] * (jj + 0.5) < c
        m = np.where(inside, BLOCK, LIT).astype(np.float32)
        pairs_a, pairs_b = [], []
        for j in range(lo, hi):
            for i in range(lo, hi):
                for t in (0.25, 0.5, 0.75):
                    if inside[j, i] != inside[j - 1, i]:  # side y = j between (i, j-1) and (i, j)
                        pairs_a.append(((i + t) / W, j / W))
                        pairs_b.append(((i + t) / W, (j - eps) / W))
                    if inside[j, i] != inside[j, i - 1]:  # side x = i
                        pairs_a.append((i / W, (j + t) / W))
                        pairs_b.append(((i - eps) / W, (j + t) / W))
        fa = np.array([(u, v, 0.9) for u, v in pairs_a], np.float32)
        fb = np.array([(u, v, 0.9) for u, v in pairs_b], np.float32)
        va, vb = oracle.rsmss(m, fa, p), oracle.rsmss(m, fb, p)
        # the two sides really are a lit and a shadowed texel
        assert np.all(oracle.shadow_map(m, fa, p) != oracle.shadow_map(m, fb, p))
        # |d nrd / d f| <= 1 per axis: the values may differ by eps, not more
        assert np.max(np.abs(va - vb)) <= 2 * eps, theta
        assert np.any((va > 0) & (va < 1))
        checked += len(fa)
    assert checked > 1000


# --------------------------------------------------------------------------
# RPCF: the correctly rounded exact mean of its terms
# --------------------------------------------------------------------------

def test_rpcf_is_the_rounded_exact_mean():
    """The box average is defined as the exact mean of the (2r+1)^2 binary32
    RSMSS terms rounded to binary32; the oracle's binary64 sum stays within
    5e-13 of it, so its result is the correctly rounded exact mean except at
    a near-tie.  Terms come from r = 0 evaluations of fragments shifted by
    whole texels, with sub-texel positions that survive the shift exactly."""
    from fractions import Fraction
    m, fr = _random_scene(17, W=32, n_rect=8)
    m = np.ascontiguousarray(m[:32, :32])
    rng = np.random.default_rng(5)
    k = 200
    i = rng.integers(0, 32, k)
    j = rng.integers(0, 32, k)
    # fractions with bits down to 2^-18 (exact in binary32 for texels < 32)
    fx = rng.integers(0, 1 << 18, k) / float(1 << 18)
    fy = rng.integers(0, 1 << 18, k) / float(1 << 18)
    fr = np.stack([(i + fx) / 32, (j + fy) / 32, fr[:k, 2]], 1).astype(np.float32)
    for r in (1, 3):
        p = params(32, bias=1e-4, max_dist=16, radius=r)
        got = oracle.rsmss(m, fr, p)
        p0 = dict(p, kernel_radius=0)
        terms = []
        for a in range(-r, r + 1):
            for b in range(-r, r + 1):
                sh = fr.copy()
                sh[:, 0] = fr[:, 0] + np.float32(a / 32)
                sh[:, 1] = fr[:, 1] + np.float32(b / 32)
                terms.append(oracle.rsmss(m, sh, p0))
        terms = np.array(terms)
        M = (2 * r + 1) ** 2
        for q in range(k):
            exact = sum(Fraction(float(t)) for t in terms[:, q]) / M
            g = float(got[q])
            ulp = float(np.spacing(np.float32(g))) if g > 0 else 2.0 ** -149
            assert abs(Fraction(g) - exact) <= Fraction(ulp) / 2 + Fraction(1, 10 ** 12), (r, q)
        assert np.any((got > 0) & (got < 1))
