"""CPU oracle for the RBSM / RSMSS per-fragment shadow pass (arXiv 1711.07793).

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  The product library
(``paper_1711_07793_amd``) never imports, links or calls it, and the two share
no code.

The arithmetic lives in ``rbsm_oracle.c`` (plain single-threaded C, binary32 in
the paper's listing order, built with ``-ffp-contract=off``); this module only
marshals numpy arrays through ctypes.  A second, independently structured
implementation (``tests/stencil_rbsm.py``, whole-map numpy array operations)
exists only to cross-check the C oracle on exhaustive tiny maps.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librbsm_oracle.so")
_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("pitch", ctypes.c_int64),
                ("depth_bias", ctypes.c_float), ("max_dist", ctypes.c_int32),
                ("kernel_radius", ctypes.c_int32)]


class Detail(ctypes.Structure):
    _fields_ = [("s", ctypes.c_float), ("d", ctypes.c_float * 3), ("rd", ctypes.c_int32 * 4),
                ("nrd", ctypes.c_float * 4), ("path", ctypes.c_int32), ("vis", ctypes.c_float)]


def build() -> str:
    """Compile the oracle with gcc (binary32, no FMA contraction, no fast-math)."""
    src = os.path.join(_HERE, "rbsm_oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", _LIB_PATH, src, "-lm"]
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
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    P = ctypes.POINTER(_Params)
    for name in ("oracle_shadow_map", "oracle_rbsm_hard", "oracle_rsmss"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, i64, P, vp]
        fn.restype = ctypes.c_int
    lib.oracle_detail_one.argtypes = [vp, vp, P, ctypes.c_int, ctypes.POINTER(Detail)]
    lib.oracle_detail_one.restype = ctypes.c_int
    lib.oracle_multi.argtypes = [vp, i64, vp, vp, i64, P, ctypes.c_int, vp, vp, vp]
    lib.oracle_multi.restype = ctypes.c_int
    lib.oracle_margin_one.argtypes = [vp, vp, P, ctypes.c_int]
    lib.oracle_margin_one.restype = ctypes.c_double
    lib.oracle_set_touch.argtypes = [vp]
    lib.oracle_set_touch.restype = None
    lib.oracle_fetch_count.argtypes = []
    lib.oracle_fetch_count.restype = ctypes.c_int64
    lib.oracle_composite.argtypes = [i64, ctypes.c_int, vp, vp, vp, vp]
    lib.oracle_composite.restype = ctypes.c_int
    d = ctypes.c_double
    lib.oracle_raster.argtypes = [vp, ctypes.c_int, d, d, d, ctypes.c_int, ctypes.c_int, i64, vp]
    lib.oracle_raster.restype = ctypes.c_int
    lib.oracle_raster_texels.argtypes = [vp, ctypes.c_int, d, d, d, ctypes.c_int, ctypes.c_int, vp, vp, i64, vp]
    lib.oracle_raster_texels.restype = ctypes.c_int
    _lib = lib
    return lib


def _params(p: dict) -> _Params:
    return _Params(int(p["width"]), int(p["height"]), int(p.get("pitch", p["width"])),
                   float(p.get("depth_bias", 0.0)), int(p.get("max_dist", 16)),
                   int(p.get("kernel_radius", 0)))


def _c(a: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _check(st: int, what: str):
    if st != 0:
        raise ValueError(f"{what}: oracle rejected the input (status {st})")


def shadow_map(map_: np.ndarray, frags: np.ndarray, params: dict) -> np.ndarray:
    """Plain shadow mapping, Eq. 1: uint8 [N], 0 = shadow, 1 = lit."""
    m, f = _c(map_, np.float32), _c(frags, np.float32).reshape(-1, 3)
    out = np.empty(f.shape[0], dtype=np.uint8)
    p = _params(params)
    _check(_load().oracle_shadow_map(m.ctypes.data, f.ctypes.data, f.shape[0], ctypes.byref(p),
                                     out.ctypes.data), "shadow_map")
    return out


def rbsm_hard(map_: np.ndarray, frags: np.ndarray, params: dict) -> np.ndarray:
    """Hard RBSM (silhouette recovery, Listings 1-4): uint8 [N], 0 = shadow, 1 = lit."""
    m, f = _c(map_, np.float32), _c(frags, np.float32).reshape(-1, 3)
    out = np.empty(f.shape[0], dtype=np.uint8)
    p = _params(params)
    _check(_load().oracle_rbsm_hard(m.ctypes.data, f.ctypes.data, f.shape[0], ctypes.byref(p),
                                    out.ctypes.data), "rbsm_hard")
    return out


def rsmss(map_: np.ndarray, frags: np.ndarray, params: dict) -> np.ndarray:
    """RSMSS (filtering, Listings 1-3 and 5), RPCF box average when kernel_radius > 0: float32 [N]."""
    m, f = _c(map_, np.float32), _c(frags, np.float32).reshape(-1, 3)
    out = np.empty(f.shape[0], dtype=np.float32)
    p = _params(params)
    _check(_load().oracle_rsmss(m.ctypes.data, f.ctypes.data, f.shape[0], ctypes.byref(p),
                                out.ctypes.data), "rsmss")
    return out


def detail(map_: np.ndarray, frag, params: dict, hard: bool) -> Detail:
    """All intermediate values of one fragment (s, d, rd, nrd, path, vis)."""
    m = _c(map_, np.float32)
    f = _c(np.asarray(frag, dtype=np.float32).reshape(3), np.float32)
    out = Detail()
    p = _params(params)
    _check(_load().oracle_detail_one(m.ctypes.data, f.ctypes.data, ctypes.byref(p), 1 if hard else 0,
                                     ctypes.byref(out)), "detail")
    return out


def multi(maps: np.ndarray, map_index: np.ndarray, frags: np.ndarray, params: dict, hard: bool):
    """Evaluate fragment k on map ``maps[map_index[k]]`` (a stack of equal maps).

    Returns (vis float32 [N], rd int32 [N, 4], nrd float32 [N, 4])."""
    ms = _c(maps, np.float32)
    stride = ms.shape[1] * ms.shape[2]
    idx = _c(map_index, np.int32)
    f = _c(frags, np.float32).reshape(-1, 3)
    n = f.shape[0]
    vis = np.empty(n, np.float32)
    rd = np.empty((n, 4), np.int32)
    nrd = np.empty((n, 4), np.float32)
    p = _params(params)
    _check(_load().oracle_multi(ms.ctypes.data, stride, idx.ctypes.data, f.ctypes.data, n,
                                ctypes.byref(p), 1 if hard else 0, vis.ctypes.data, rd.ctypes.data,
                                nrd.ctypes.data), "multi")
    return vis, rd, nrd


def margin(map_: np.ndarray, frag, params: dict, hard: bool) -> float:
    """Binary64 distance of one fragment to its nearest decision boundary."""
    m = _c(map_, np.float32)
    f = _c(np.asarray(frag, dtype=np.float32).reshape(3), np.float32)
    p = _params(params)
    return float(_load().oracle_margin_one(m.ctypes.data, f.ctypes.data, ctypes.byref(p), 1 if hard else 0))


def touched_texels(map_: np.ndarray, frags: np.ndarray, params: dict, hard: bool):
    """Run the pass with read instrumentation.

    Returns (touch uint8 [H, W] marking every texel read, number of reads)."""
    H, W = int(params["height"]), int(params["width"])
    touch = np.zeros((H, W), np.uint8)
    lib = _load()
    lib.oracle_set_touch(touch.ctypes.data)
    try:
        if hard:
            rbsm_hard(map_, frags, params)
        else:
            rsmss(map_, frags, params)
        reads = int(lib.oracle_fetch_count())
    finally:
        lib.oracle_set_touch(None)
    return touch, reads


def composite(vis: list, weights) -> np.ndarray:
    """Multi-light compositing: float32 [N] = sum over lights in order of
    weight * visibility (binary32 products, then sums).  Each entry of ``vis``
    is a uint8 hard mask or a float32 visibility array of the same length."""
    arrs = [np.ascontiguousarray(v) for v in vis]
    n = arrs[0].shape[0] if arrs else 0
    if not 1 <= len(arrs) <= 8 or any(a.shape != (n,) for a in arrs):
        raise ValueError("composite: need 1..8 arrays of one length")
    hard = np.array([1 if a.dtype == np.uint8 else 0 for a in arrs], np.int32)
    arrs = [a if a.dtype == np.uint8 else a.astype(np.float32) for a in arrs]
    w = np.ascontiguousarray(weights, np.float32)
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    out = np.empty(n, np.float32)
    _check(_load().oracle_composite(n, len(arrs), ptrs, hard.ctypes.data, w.ctypes.data, out.ctypes.data),
           "composite")
    return out


# Primitive record of oracle_raster (112 bytes; the same field layout as the
# generator's export).
PRIM_DTYPE = np.dtype([("kind", "<i4"), ("nv", "<i4"), ("x", "<f8", (4,)), ("y", "<f8", (4,)),
                       ("nx", "<f8"), ("ny", "<f8"), ("o", "<f8"), ("w", "<f8"), ("depth", "<f4"),
                       ("pad", "<i4")])


def raster(prims: np.ndarray, receiver, width: int, height: int) -> np.ndarray:
    """Shadow-map rasterization: float32 [height, width] of the nearest
    surface at each texel centre (receiver plane or covering primitive)."""
    p = np.ascontiguousarray(prims, dtype=PRIM_DTYPE)
    out = np.empty((height, width), np.float32)
    r0, ru, rv = receiver
    _check(_load().oracle_raster(p.ctypes.data if len(p) else None, len(p), r0, ru, rv, width, height, width,
                                 out.ctypes.data), "raster")
    return out


def raster_texels(prims: np.ndarray, receiver, width: int, height: int, ti: np.ndarray, tj: np.ndarray) -> np.ndarray:
    """``raster`` at chosen texels (column ti[k], row tj[k]): float32 [count]."""
    p = np.ascontiguousarray(prims, dtype=PRIM_DTYPE)
    i32 = np.ascontiguousarray(ti, np.int32)
    j32 = np.ascontiguousarray(tj, np.int32)
    out = np.empty(len(i32), np.float32)
    r0, ru, rv = receiver
    _check(_load().oracle_raster_texels(p.ctypes.data if len(p) else None, len(p), r0, ru, rv, width, height,
                                        i32.ctypes.data, j32.ctypes.data, len(i32), out.ctypes.data),
           "raster_texels")
    return out
