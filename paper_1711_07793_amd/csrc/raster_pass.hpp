// Shadow-map rasterization on the device: the light pass whose depth map the
// RBSM pass consumes (Sec. 2 takes it as given).  Included once, by rbsm.hip.
//
// A texel (i, j) samples its centre ((i + 0.5) / W, (j + 0.5) / H) in texture
// coordinates; it holds the nearest surface there: the receiver plane
// r0 + ru (u - 0.5) + rv (v - 0.5) (binary64, rounded to binary32) unless a
// primitive covering the centre has a smaller depth; among equal depths
// (+0 and -0 compare equal) the plane wins, then the primitive of lowest
// index.  A convex counter-clockwise polygon covers a point when no edge
// function (b - a) x (p - a) is negative and every zero lies on an edge that
// owns ties (one running downwards, or horizontally to the left: the
// top-left rule); a slab covers o <= nx u + ny v < o + w.  All coverage
// arithmetic is binary64 without contraction, so decisions are reproducible
// exactly.
//
// One workgroup per texel tile: 32 x 32 (256 threads), 16 x 16 (64 threads)
// on maps under 2^22 texels so the grid still fills the GPU, 64 x 64 on maps
// of 2^25 texels or more to amortize the classification.  Each primitive is
// classified against the tile's rectangle of texel centres, with a margin far
// above the binary64 rounding of the edge functions: covering none (so every
// per-texel test would fail), covering every one (every test would pass), or
// partial.  The covering ones reduce to one tile-wide nearest depth; only the
// partial ones, listed in LDS, are tested per texel.  The winner among equal
// depths is decided by primitive index, so the result does not depend on the
// order of either list.  A thread writes its 4 texels of a row with one
// 16-byte store when rows start 16-byte aligned.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbsm.h"
#include "tile_pass.hpp"

namespace rbsm {

constexpr int kRasT = 256;      // threads per workgroup (32 x 32 and 64 x 64 tiles)
constexpr int kRasTile = 32;    // tile side in texels on mid-size maps; a thread owns 4 texels of a row
constexpr int kRasList = 2048;  // primitives listed per tile before falling back to all

__device__ __forceinline__ double edge_value(double ax, double ay, double bx, double by, double px, double py) {
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

__device__ __forceinline__ bool covers(const rbsm_prim &q, double px, double py) {
    if (q.kind == 1) {
        const double t = q.nx * px + q.ny * py;
        return t >= q.o && t < q.o + q.w;
    }
    if (q.kind != 0 || q.nv < 3 || q.nv > 4) return false;
    for (int e = 0; e < q.nv; ++e) {
        const int f = e + 1 == q.nv ? 0 : e + 1;
        const double v = edge_value(q.x[e], q.y[e], q.x[f], q.y[f], px, py);
        if (v < 0.0) return false;
        if (v == 0.0) {
            const double dy = q.y[f] - q.y[e], dx = q.x[f] - q.x[e];
            if (!(dy < 0.0 || (dy == 0.0 && dx < 0.0))) return false;
        }
    }
    return true;
}

// May q cover a texel centre in [u0, u1] x [v0, v1]?  Bounds grown by `pad`
// (a texel) so rounding never drops a covering primitive.
__device__ __forceinline__ bool may_touch(const rbsm_prim &q, double u0, double u1, double v0, double v1, double pad) {
    if (q.kind == 1) {
        const double t00 = q.nx * u0 + q.ny * v0, t10 = q.nx * u1 + q.ny * v0;
        const double t01 = q.nx * u0 + q.ny * v1, t11 = q.nx * u1 + q.ny * v1;
        const double lo = fmin(fmin(t00, t10), fmin(t01, t11)), hi = fmax(fmax(t00, t10), fmax(t01, t11));
        return hi + pad >= q.o && lo - pad < q.o + q.w;
    }
    if (q.kind != 0 || q.nv < 3 || q.nv > 4) return false;
    double xmin = q.x[0], xmax = q.x[0], ymin = q.y[0], ymax = q.y[0];
    for (int e = 1; e < q.nv; ++e) {
        xmin = fmin(xmin, q.x[e]);
        xmax = fmax(xmax, q.x[e]);
        ymin = fmin(ymin, q.y[e]);
        ymax = fmax(ymax, q.y[e]);
    }
    return xmax + pad >= u0 && xmin - pad <= u1 && ymax + pad >= v0 && ymin - pad <= v1;
}

// How q meets the texel centres of [u0, u1] x [v0, v1] (all in [0, 1]):
// 0 none, 2 every one, 1 maybe some.  An edge function is affine, so its exact
// extremes over the rectangle are at corners; binary64 evaluation errs by well
// under 2^-50 times the scale below, so corner values beyond 2^-40 times that
// scale fix the sign of every centre's binary64 value.  Slabs likewise on
// nx u + ny v.  Answer 1 is always safe: q is then tested texel by texel.
__device__ __forceinline__ int tile_cover(const rbsm_prim &q, double u0, double u1, double v0, double v1) {
    const double k = 0x1p-40;
    if (q.kind == 1) {
        const double t00 = q.nx * u0 + q.ny * v0, t10 = q.nx * u1 + q.ny * v0;
        const double t01 = q.nx * u0 + q.ny * v1, t11 = q.nx * u1 + q.ny * v1;
        const double lo = fmin(fmin(t00, t10), fmin(t01, t11)), hi = fmax(fmax(t00, t10), fmax(t01, t11));
        const double m = k * (fabs(q.nx) + fabs(q.ny));
        const double end = q.o + q.w;
        if (hi + m < q.o || lo - m >= end) return 0;
        return lo - m >= q.o && hi + m < end ? 2 : 1;
    }
    if (q.kind != 0 || q.nv < 3 || q.nv > 4) return 0;
    bool all = true;
    for (int e = 0; e < q.nv; ++e) {
        const int f = e + 1 == q.nv ? 0 : e + 1;
        const double ax = q.x[e], ay = q.y[e], bx = q.x[f], by = q.y[f];
        const double m = k * (fabs(bx - ax) * (1.0 + fabs(ay)) + fabs(by - ay) * (1.0 + fabs(ax)));
        const double e00 = edge_value(ax, ay, bx, by, u0, v0), e10 = edge_value(ax, ay, bx, by, u1, v0);
        const double e01 = edge_value(ax, ay, bx, by, u0, v1), e11 = edge_value(ax, ay, bx, by, u1, v1);
        if (fmax(fmax(e00, e10), fmax(e01, e11)) < -m) return 0;  // negative at every centre
        all = all && fmin(fmin(e00, e10), fmin(e01, e11)) > m;    // false on NaN
    }
    return all ? 2 : 1;
}

// Depth z of primitive k beats the current (d, from primitive idx; -1 is the
// receiver plane): smaller, or equal and of lower index.
__device__ __forceinline__ bool beats(float z, int k, float d, int idx) { return z < d || (z == d && k < idx); }

template <int TS, int NT>
__global__ __launch_bounds__(NT) void raster_kernel(const rbsm_prim *__restrict__ prims, int n, double r0,
                                                       double ru, double rv, int W, int H, int64_t pitch,
                                                       float *__restrict__ map, int tiles_x, bool vec) {
    __shared__ int s_list[kRasList];  // partly covering primitives
    __shared__ int s_full[kRasList];  // primitives covering every centre
    __shared__ int s_count, s_nfull;
    const int t = threadIdx.x;
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int ty = (int)(tile / tiles_x), tx = (int)(tile - (int64_t)ty * tiles_x);
    const int i0 = tx * TS, j0 = ty * TS;
    const int i1 = min(i0 + TS, W) - 1, j1 = min(j0 + TS, H) - 1;
    const double u0 = (i0 + 0.5) / W, u1 = (i1 + 0.5) / W;
    const double v0 = (j0 + 0.5) / H, v1 = (j1 + 0.5) / H;
    const double pad = 1.0 / (double)(W < H ? W : H);
    if (t == 0) {
        s_count = 0;
        s_nfull = 0;
    }
    __syncthreads();
    for (int k = t; k < n; k += NT) {
        const rbsm_prim &q = prims[k];
        if (!may_touch(q, u0, u1, v0, v1, pad)) continue;
        const int c = tile_cover(q, u0, u1, v0, v1);
        if (c == 0) continue;
        int *list = c == 2 ? s_full : s_list;
        const int slot = atomicAdd(c == 2 ? &s_nfull : &s_count, 1);
        if (slot < kRasList) list[slot] = k;
    }
    __syncthreads();
    // too many to list: test every primitive at every texel
    const bool all = s_count > kRasList || s_nfull > kRasList;
    const int m = all ? n : s_count, mf = all ? 0 : s_nfull;

    // nearest of the covering primitives, ties by index (order-free)
    float fz = __builtin_inff();
    int fk = INT32_MAX;
    for (int c = 0; c < mf; ++c) {
        const int k = s_full[c];
        const float z = prims[k].depth;
        if (beats(z, k, fz, fk)) {
            fz = z;
            fk = k;
        }
    }
    // each thread resolves 4 texels of a row, NT / (TS / 4) rows apart
    constexpr int RP = NT / (TS / 4);  // rows per pass
    const int col = i0 + (t % (TS / 4)) * 4;
    for (int row = j0 + t / (TS / 4); row <= j1; row += RP) {
        const double py = (row + 0.5) / H;
        float d[4];
        int di[4];
        double px[4];
        for (int e = 0; e < 4; ++e) {
            px[e] = (col + e + 0.5) / W;
            d[e] = (float)(r0 + ru * (px[e] - 0.5) + rv * (py - 0.5));
            di[e] = -1;
            if (fk != INT32_MAX && beats(fz, fk, d[e], di[e])) {
                d[e] = fz;
                di[e] = fk;
            }
        }
        for (int c = 0; c < m; ++c) {
            const int k = __builtin_amdgcn_readfirstlane(all ? c : s_list[c]);
            const rbsm_prim &q = prims[k];
            const float z = q.depth;
            for (int e = 0; e < 4; ++e)
                if (col + e <= i1 && beats(z, k, d[e], di[e]) && covers(q, px[e], py)) {
                    d[e] = z;
                    di[e] = k;
                }
        }
        float *dst = map + (int64_t)row * pitch + col;
        if (vec && col + 3 <= i1) {  // one 16-byte store
            *(float4 *)dst = make_float4(d[0], d[1], d[2], d[3]);
        } else {
            for (int e = 0; e < 4; ++e)
                if (col + e <= i1) dst[e] = d[e];
        }
    }
}

inline void launch_raster(const rbsm_prim *prims, int n, double r0, double ru, double rv, int W, int H, int64_t pitch,
                          float *map, hipStream_t stream) {
    // tiles sized so the grid has several workgroups per resident slot: 16 x 16
    // (64 threads) on maps under 2^22 texels, 64 x 64 on maps of 2^25 or more
    // (which amortizes the classification), else 32 x 32
    const int64_t area = (int64_t)W * H;
    const int ts = area < ((int64_t)1 << 22) ? 16 : (area >= ((int64_t)1 << 25) ? 64 : kRasTile);
    const int tiles_x = (W + ts - 1) / ts, tiles_y = (H + ts - 1) / ts;
    const dim3 grid((unsigned)((int64_t)tiles_x * tiles_y));
    // rows start 16-byte aligned: a thread's 4 texels (columns 4k .. 4k+3) are one float4
    const bool vec = ((uintptr_t)map & 15u) == 0 && (pitch & 3) == 0;
    if (ts == 16)
        hipLaunchKernelGGL((raster_kernel<16, 64>), grid, dim3(64), 0, stream, prims, n, r0, ru, rv, W, H, pitch, map,
                           tiles_x, vec);
    else if (ts == 64)
        hipLaunchKernelGGL((raster_kernel<64, kRasT>), grid, dim3(kRasT), 0, stream, prims, n, r0, ru, rv, W, H,
                           pitch, map, tiles_x, vec);
    else
        hipLaunchKernelGGL((raster_kernel<kRasTile, kRasT>), grid, dim3(kRasT), 0, stream, prims, n, r0, ru, rv, W,
                           H, pitch, map, tiles_x, vec);
}

}  // namespace rbsm
