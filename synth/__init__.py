"""Seeded synthetic inputs for the RBSM shadow pass.

This package holds none of the method's arithmetic.  It produces light-space
depth maps (the light pass the paper takes as given, Sec. 2) and light-space
camera fragments (the varying ``p`` of the RBSM listing, Sec. 3), both as
numpy arrays, deterministically from a seed.  The CPU oracle and the GPU path
both consume what it returns.

Workload recipes (sizes and distributions) follow the five evaluation
configurations of the project: a single rotated quad over a flat receiver
(512^2 map, 65,536 uniform fragments), random-triangle scenes over a tilted
receiver seen by a perspective camera (2048^2 map, 1920x1080), and the same
with a thin-bar fence (4096^2 map, 3840x2160).  They stand in for the paper's
Fence and QuadBot scenes (Sec. 5), whose models are not available.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build() -> str:
    """Compile the generator with gcc into ``synth/libsynth.so``."""
    src = os.path.join(_HERE, "synth.c")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", _LIB_PATH, src, "-lm"]
    subprocess.run(cmd, check=True)
    global _lib
    _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    lib.synth_scene_quad.restype = vp
    lib.synth_scene_quad.argtypes = [u64, ctypes.c_int, ctypes.c_int]
    lib.synth_scene_tris.restype = vp
    lib.synth_scene_tris.argtypes = [u64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.synth_scene_free.argtypes = [vp]
    lib.synth_scene_free.restype = None
    lib.synth_scene_raster.argtypes = [vp, vp, i64]
    lib.synth_scene_raster.restype = ctypes.c_int
    lib.synth_scene_count.argtypes = [vp]
    lib.synth_scene_count.restype = ctypes.c_int
    lib.synth_frags_uniform.argtypes = [u64, i64, ctypes.c_float, vp]
    lib.synth_frags_uniform.restype = None
    lib.synth_frags_camera.argtypes = [vp, u64, ctypes.c_int, ctypes.c_int, ctypes.c_double, vp]
    lib.synth_frags_camera.restype = ctypes.c_int
    lib.synth_frags_camera_rows.argtypes = [vp, u64, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_int, vp]
    lib.synth_frags_camera_rows.restype = ctypes.c_int
    lib.synth_uniform_f32.argtypes = [u64, i64, vp]
    lib.synth_uniform_f32.restype = None
    lib.synth_scene_export.argtypes = [vp, vp, ctypes.c_int, vp]
    lib.synth_scene_export.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# One primitive of a blocker scene: kind 0 is a convex counter-clockwise
# polygon of nv (3 or 4) vertices in texture coordinates, kind 1 a slab
# o <= nx*u + ny*v < o + w; depth is the blocker's constant light-space depth.
PRIM_DTYPE = np.dtype([("kind", "<i4"), ("nv", "<i4"), ("x", "<f8", (4,)), ("y", "<f8", (4,)),
                       ("nx", "<f8"), ("ny", "<f8"), ("o", "<f8"), ("w", "<f8"), ("depth", "<f4"),
                       ("pad", "<i4")])
assert PRIM_DTYPE.itemsize == 112


class Scene:
    """A blocker scene in light space (owns the C object)."""

    def __init__(self, handle: int, width: int, height: int):
        self._h = handle
        self.width = width
        self.height = height

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.synth_scene_free(self._h)
            self._h = None

    @property
    def n_prims(self) -> int:
        return _load().synth_scene_count(self._h)

    def raster(self, pitch: int | None = None) -> np.ndarray:
        """Depth map as float32 [height, pitch] (columns >= width are padding, 0)."""
        pitch = self.width if pitch is None else pitch
        out = np.zeros((self.height, pitch), dtype=np.float32)
        _load().synth_scene_raster(self._h, _ptr(out), pitch)
        return out

    def primitives(self):
        """The scene's primitives as a structured array (PRIM_DTYPE, 112 bytes
        a record) and its receiver plane (r0, ru, rv)."""
        n = self.n_prims
        out = np.zeros(max(n, 1), dtype=PRIM_DTYPE)
        rec = np.zeros(3, dtype=np.float64)
        _load().synth_scene_export(self._h, out.ctypes.data, n, rec.ctypes.data)
        return out[:n], (float(rec[0]), float(rec[1]), float(rec[2]))

    def camera_fragments(self, seed: int, width: int, height: int, vfov_deg: float = 40.0) -> np.ndarray:
        """Perspective-camera fragments, float32 [width*height, 3] = (u, v, z), screen row-major."""
        out = np.empty((width * height, 3), dtype=np.float32)
        st = _load().synth_frags_camera(self._h, seed, width, height, vfov_deg, _ptr(out))
        if st != 0:
            raise RuntimeError(f"camera footprint left the map (status {st})")
        return out


    def camera_rows(self, seed: int, width: int, height: int, r0: int, r1: int,
                    vfov_deg: float = 40.0) -> np.ndarray:
        """Rows [r0, r1) of the camera image of ``camera_fragments`` (same values)."""
        out = np.empty(((r1 - r0) * width, 3), dtype=np.float32)
        st = _load().synth_frags_camera_rows(self._h, seed, width, height, vfov_deg, r0, r1, _ptr(out))
        if st != 0:
            raise RuntimeError(f"camera rows failed (status {st})")
        return out


def quad_scene(seed: int, width: int, height: int) -> Scene:
    return Scene(_load().synth_scene_quad(seed, width, height), width, height)


def triangle_scene(seed: int, width: int, height: int, n_tris: int, fence: bool = False) -> Scene:
    return Scene(_load().synth_scene_tris(seed, width, height, n_tris, 1 if fence else 0), width, height)


def uniform_fragments(seed: int, n: int, z: float) -> np.ndarray:
    """n fragments, (u, v) i.i.d. uniform on [0,1)^2, constant depth z; float32 [n, 3]."""
    out = np.empty((n, 3), dtype=np.float32)
    _load().synth_frags_uniform(seed, n, z, _ptr(out))
    return out


def uniform_floats(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float32)
    _load().synth_uniform_f32(seed, n, _ptr(out))
    return out


HARD, RSMSS = "hard", "rsmss"


def make_config(k: int, seed: int, small: bool = False) -> dict:
    """Inputs of workload ``k`` (1..3) for ``seed``.

    Returns a dict with ``map`` (float32 [H, W]), ``frags`` (float32 [N, 3]),
    ``params`` (width, height, pitch, depth_bias, max_dist, kernel_radius) and
    ``mode`` (``"hard"`` or ``"rsmss"``).  ``small=True`` shrinks the camera
    resolution 8x per axis (for quick tests) while keeping the scene.
    """
    if k == 1:
        W = H = 512
        sc = quad_scene(seed, W, H)
        m = sc.raster()
        n = 65536 if not small else 8192
        fr = uniform_fragments(seed ^ 0x5EED_F4A6, n, np.float32(0.9))
        return dict(map=m, frags=fr, mode=HARD, scene=sc,
                    params=dict(width=W, height=H, pitch=W, depth_bias=1e-4, max_dist=16, kernel_radius=0,
                                view_width=0),
                    name="quad512_uniform65536_hard")
    if k == 2:
        W = H = 2048
        sc = triangle_scene(seed, W, H, 64, fence=False)
        m = sc.raster()
        sw, sh = (1920, 1080) if not small else (240, 135)
        fr = sc.camera_fragments(seed ^ 0xCA3E_2A00, sw, sh)
        return dict(map=m, frags=fr, mode=HARD, scene=sc,
                    params=dict(width=W, height=H, pitch=W, depth_bias=1e-4, max_dist=32, kernel_radius=0,
                                view_width=sw),
                    name=f"tri64_map2048_view{sw}x{sh}_hard")
    if k == 3:
        W = H = 4096
        sc = triangle_scene(seed, W, H, 256, fence=True)
        m = sc.raster()
        sw, sh = (3840, 2160) if not small else (480, 270)
        fr = sc.camera_fragments(seed ^ 0xCA3E_3A00, sw, sh)
        radius = 3 + int(uniform_floats(seed ^ 0x3AD1_0005, 1)[0] * 13)
        return dict(map=m, frags=fr, mode=RSMSS, scene=sc, light_radius=radius,
                    params=dict(width=W, height=H, pitch=W, depth_bias=1e-4, max_dist=16, kernel_radius=0,
                                view_width=sw),
                    name=f"tri256fence_map4096_view{sw}x{sh}_rsmss")
    raise ValueError(f"unknown workload {k}")


def make_batched(seed: int, small: bool = False) -> dict:
    """Batched workload: 16 shadow maps (a directional light's 4 cascades of
    8192^2, 4096^2, 2048^2, 1024^2 and 12 spot lights of 1024^2..4096^2, each a
    random-triangle scene) and 8 views (two each of 1280x720, 1920x1080,
    2560x1440, 3840x2160).  Each view's rows are split among the 4 cascades
    (Dirichlet fractions, near rows to the finest cascade) and 2 spot lights
    each cover a band of U(0.3, 1.0) of its rows: 48 jobs of uneven size.
    Cascade jobs are hard (MAXDIST 32 on the two finest maps, 16 after),
    spot jobs RSMSS radius 0 (MAXDIST 16); depth bias 1e-4.  ``small``
    divides every map side by 16 and every view side by 8 (test size).

    Returns dict(maps=[float32 [S, S]], jobs=[dict(map=i, frags=[N, 3],
    params=..., mode=0/1, view=v, rows=(r0, r1))]).
    """
    rng = np.random.default_rng(seed)
    div_m, div_v = (16, 8) if small else (1, 1)
    cascade = [8192, 4096, 2048, 1024]
    spot = [int(rng.choice([1024, 2048, 4096])) for _ in range(12)]
    sizes = [s // div_m for s in cascade + spot]
    scenes = [triangle_scene(seed * 100 + i, s, s, 64, fence=False) for i, s in enumerate(sizes)]
    maps = [sc.raster() for sc in scenes]
    views = [(1280, 720), (1280, 720), (1920, 1080), (1920, 1080), (2560, 1440), (2560, 1440),
             (3840, 2160), (3840, 2160)]
    jobs = []
    for v, (ws, hs) in enumerate(views):
        ws, hs = ws // div_v, hs // div_v
        cam_seed = seed * 1000 + v
        frac = rng.dirichlet([2.0, 2.0, 2.0, 2.0])
        cuts = np.concatenate([[0], np.round(np.cumsum(frac) * hs).astype(int)])
        cuts[-1] = hs
        # rows run far (top) to near (bottom): the nearest rows use cascade 0
        for c in range(4):
            r1, r0 = hs - cuts[c], hs - cuts[c + 1]
            if r1 <= r0:
                continue
            S = sizes[c]
            fr = scenes[c].camera_rows(cam_seed, ws, hs, r0, r1)
            jobs.append(dict(map=c, frags=fr, mode=0, view=v, rows=(r0, r1),
                             params=dict(width=S, height=S, pitch=S, depth_bias=1e-4,
                                         max_dist=32 if c < 2 else 16, kernel_radius=0, view_width=ws)))
        for sl in rng.choice(12, size=2, replace=False):
            m_idx = 4 + int(sl)
            cover = rng.uniform(0.3, 1.0)
            nr = max(1, int(round(cover * hs)))
            r0 = int(rng.integers(0, hs - nr + 1))
            S = sizes[m_idx]
            fr = scenes[m_idx].camera_rows(cam_seed, ws, hs, r0, r0 + nr)
            jobs.append(dict(map=m_idx, frags=fr, mode=1, view=v, rows=(r0, r0 + nr),
                             params=dict(width=S, height=S, pitch=S, depth_bias=1e-4, max_dist=16,
                                         kernel_radius=0, view_width=ws)))
    return dict(maps=maps, jobs=jobs, views=[(w // div_v, h // div_v) for w, h in views])
