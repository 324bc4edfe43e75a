"""A second RBSM implementation, structured as whole-map array stencils.

Test aid only: it cross-checks the C oracle on exhaustive tiny maps.  Where the
oracle walks one fragment at a time through the listings' branches, this module
works on binary test maps S (one per map, all fragments at one depth, so the
shadow test is a per-texel quantity), computes the neighbour-discontinuity bit
masks of every texel with shifted-array comparisons, runs all traversals of all
texels at once as "first stopping step" searches over k = 1..MAXDIST, and
evaluates the visibility functions in their select-only form (no shape
branches).  Map borders use clamp-to-edge, realised here by edge padding.

Bits: L = 1, R = 2, T (+y) = 4, B (-y) = 8.
"""
from __future__ import annotations

import numpy as np

L, R, T, B = 1, 2, 4, 8


def _masks(Sp: np.ndarray) -> np.ndarray:
    """Discontinuity bits of every interior texel of the padded stack Sp [n, h, w]
    (the outermost ring is dropped)."""
    c = Sp[:, 1:-1, 1:-1]
    m = np.zeros(c.shape, np.int8)
    m |= np.where(Sp[:, 1:-1, :-2] != c, L, 0)
    m |= np.where(Sp[:, 1:-1, 2:] != c, R, 0)
    m |= np.where(Sp[:, 2:, 1:-1] != c, T, 0)
    m |= np.where(Sp[:, :-2, 1:-1] != c, B, 0)
    return m


def evaluate(S: np.ndarray, map_idx: np.ndarray, ti: np.ndarray, tj: np.ndarray,
             fx: np.ndarray, fy: np.ndarray, max_dist: int, hard: bool):
    """Visibility of fragments on binary test maps.

    S: uint8 [n_maps, H, W], 1 = lit test result, 0 = shadowed.
    Fragment k lies on map map_idx[k], texel (ti[k], tj[k]) (inside the map),
    sub-texel position (fx[k], fy[k]) (float32).
    Returns (vis float32, rd int32 [N, 4] left/right/top/bottom with 0 where no
    walk ran, nrd float32 [N, 4]).
    """
    S = S.astype(np.int8)
    n_maps, H, W = S.shape
    pad = max_dist + 2
    Sp = np.pad(S, ((0, 0), (pad, pad), (pad, pad)), mode="edge")
    Mp = np.zeros_like(Sp, dtype=np.int8)
    Mp[:, 1:-1, 1:-1] = _masks(Sp)

    N = map_idx.shape[0]
    pi = ti + pad
    pj = tj + pad
    s = Sp[map_idx, pj, pi]
    m0 = Mp[map_idx, pj, pi]

    # walks: left, right, top, bottom
    dirs = [(-1, 0), (1, 0), (0, 1), (0, -1)]
    ks = np.arange(1, max_dist + 1)
    rd = np.zeros((N, 4), np.int32)
    for w, (dx, dy) in enumerate(dirs):
        qi = pi[:, None] + ks[None, :] * dx
        qj = pj[:, None] + ks[None, :] * dy
        sq = Sp[map_idx[:, None], qj, qi]
        mq = Mp[map_idx[:, None], qj, qi]
        is_end = sq != s[:, None]
        leaves = (~is_end) & ((mq & m0[:, None]) == 0)
        stops = is_end | leaves
        any_stop = stops.any(axis=1)
        first = np.argmax(stops, axis=1)  # index of the first stopping step
        k_stop = ks[first]
        end_at_stop = is_end[np.arange(N), first]
        rd[:, w] = np.where(any_stop, np.where(end_at_stop, k_stop, -k_stop), -(max_dist + 1))

    one = np.float32(1.0)

    def axis(neg, pos, f):
        ends = (neg > 0).astype(np.int32) + (pos > 0).astype(np.int32)
        an, ap = np.abs(neg), np.abs(pos)
        length = (an + ap - 1).astype(np.float32)
        length = np.where(length > 0, length, one)
        toward_pos = ap.astype(np.float32) - f
        toward_neg = (an - 1).astype(np.float32) + f
        a = np.where(pos > 0, toward_pos, toward_neg).astype(np.float32)
        val = (a / length).astype(np.float32)
        code = np.where(ends == 2, 1, np.where(ends == 0, -1, 0)).astype(np.float32)
        val = np.where(ends == 2, np.float32(0), np.where(ends == 0, one, val)).astype(np.float32)
        return val, code

    nx, cx = axis(rd[:, 0], rd[:, 1], fx.astype(np.float32))
    ny, cy = axis(rd[:, 3], rd[:, 2], fy.astype(np.float32))
    nrd = np.stack([nx, ny, cx, cy], axis=1).astype(np.float32)

    edge = m0 != 0
    sf = s.astype(np.float32)
    if hard:
        lit_edge = (cx != 1) & (cy != 1) & ~(ny < (one - nx))
        vis = np.where(s == 0, np.float32(0), np.where(edge, lit_edge.astype(np.float32), sf))
        keep = (s != 0) & edge
    else:
        dz = one - sf
        sg = one - np.float32(2) * dz
        tx = np.where(cx == 1, np.float32(0), nx).astype(np.float32)
        ty = np.where(cy == 1, np.float32(0), ny).astype(np.float32)
        v = ((dz + sg * ty).astype(np.float32) + sg * tx).astype(np.float32)
        v = np.minimum(np.maximum(v, np.float32(0)), one)
        vis = np.where(edge, v, sf)
        keep = edge
    rd = np.where(keep[:, None], rd, 0).astype(np.int32)
    nrd = np.where(keep[:, None], nrd, np.float32(0)).astype(np.float32)
    return vis.astype(np.float32), rd, nrd
