"""The seeded input generator: determinism, ranges and workload shapes."""
import numpy as np

import synth


def test_streams_are_seeded_and_uniform():
    a = synth.uniform_floats(123, 100000)
    b = synth.uniform_floats(123, 100000)
    c = synth.uniform_floats(124, 100000)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0.0 and a.max() < 1.0
    assert abs(a.mean() - 0.5) < 0.01 and abs(a.var() - 1 / 12) < 0.01
    # 24-bit grid
    assert np.all(a * 2 ** 24 == np.floor(a * 2 ** 24))


def test_quad_workload():
    c1 = synth.make_config(1, 1001)
    c2 = synth.make_config(1, 1001)
    assert np.array_equal(c1["map"], c2["map"]) and np.array_equal(c1["frags"], c2["frags"])
    m = c1["map"]
    assert m.shape == (512, 512) and m.dtype == np.float32
    blocked = m < 0.9
    side = np.sqrt(blocked.sum())
    assert 0.3 * 512 * 0.95 < side < 0.6 * 512 * 1.05
    assert np.unique(m).size == 2
    f = c1["frags"]
    assert f.shape == (65536, 3) and np.all(f[:, 2] == np.float32(0.9))


def test_triangle_camera_workload_small():
    c = synth.make_config(2, 2001, small=True)
    m, f = c["map"], c["frags"]
    assert m.shape == (2048, 2048)
    assert f.shape == (240 * 135, 3)
    assert np.all((f[:, :2] >= 0) & (f[:, :2] < 1))
    # receiver tilt: texel centres follow 0.9 + 0.05 (u - .5) + 0.03 (v - .5)
    assert abs(float(m[0, 0]) - (0.9 + 0.05 * (0.5 / 2048 - 0.5) + 0.03 * (0.5 / 2048 - 0.5))) < 1e-6 or m[0, 0] < 0.85
    assert (m < 0.85).mean() > 0.01
    # some fragments land on blockers (depth below the receiver)
    assert (f[:, 2] <= 0.8).any() and (f[:, 2] > 0.85).any()
    # screen order: neighbouring pixels are close in light space (except
    # where a ray moves between a blocker and the receiver)
    step = np.abs(np.diff(f[:240, :2], axis=0)).max(axis=1)
    assert np.median(step) < 0.01


def test_fence_workload_small():
    c = synth.make_config(3, 3001, small=True)
    m = c["map"]
    assert m.shape == (4096, 4096)
    assert c["scene"].n_prims == 256 + 32
    assert 3 <= c["light_radius"] <= 15
    assert c["frags"].shape == (480 * 270, 3)
