// Shadow-map rasterization on the device: the light pass whose depth map the
// RBSM pass consumes (Sec. 2 takes it as given).  Included once, by rbsm.hip.
//
// A texel (i, j) samples its centre ((i + 0.5) / W, (j + 0.5) / H) in texture
// coordinates; it holds the nearest surface there: the minimum of the
// receiver plane r0 + ru (u - 0.5) + rv (v - 0.5) (binary64, rounded to
// binary32) and the depth of every primitive covering the centre.  A convex
// counter-clockwise polygon covers a point when no edge function
// (b - a) x (p - a) is negative and every zero lies on an edge that owns ties
// (one running downwards, or horizontally to the left: the top-left rule); a
// slab covers o <= nx u + ny v < o + w.  All coverage arithmetic is binary64
// without contraction, so decisions are reproducible exactly.
//
// One workgroup per 32 x 32 texel tile: the primitives whose bounds (grown by
// a texel) reach the tile are listed in LDS, then each thread resolves four
// texels of a row against the list.  The minimum does not depend on the
// order of the list.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbsm.h"
#include "tile_pass.hpp"

namespace rbsm {

constexpr int kRasT = 256;      // threads per workgroup
constexpr int kRasTile = 32;    // tile side in texels; a thread owns 4 texels of a row
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

__global__ __launch_bounds__(kRasT) void raster_kernel(const rbsm_prim *__restrict__ prims, int n, double r0,
                                                       double ru, double rv, int W, int H, int64_t pitch,
                                                       float *__restrict__ map, int tiles_x) {
    __shared__ int s_list[kRasList];
    __shared__ int s_count;
    const int t = threadIdx.x;
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int ty = (int)(tile / tiles_x), tx = (int)(tile - (int64_t)ty * tiles_x);
    const int i0 = tx * kRasTile, j0 = ty * kRasTile;
    const int i1 = min(i0 + kRasTile, W) - 1, j1 = min(j0 + kRasTile, H) - 1;
    const double u0 = (i0 + 0.5) / W, u1 = (i1 + 0.5) / W;
    const double v0 = (j0 + 0.5) / H, v1 = (j1 + 0.5) / H;
    const double pad = 1.0 / (double)(W < H ? W : H);
    if (t == 0) s_count = 0;
    __syncthreads();
    for (int k = t; k < n; k += kRasT) {
        if (!may_touch(prims[k], u0, u1, v0, v1, pad)) continue;
        const int slot = atomicAdd(&s_count, 1);
        if (slot < kRasList) s_list[slot] = k;
    }
    __syncthreads();
    const int listed = s_count;
    const bool all = listed > kRasList;  // too many to list: test every primitive
    const int m = all ? n : listed;

    const int row = j0 + t / (kRasTile / 4);
    const int col = i0 + (t % (kRasTile / 4)) * 4;
    if (row > j1) return;
    const double py = (row + 0.5) / H;
    float d[4];
    double px[4];
    for (int e = 0; e < 4; ++e) {
        px[e] = (col + e + 0.5) / W;
        d[e] = (float)(r0 + ru * (px[e] - 0.5) + rv * (py - 0.5));
    }
    for (int c = 0; c < m; ++c) {
        const int k = __builtin_amdgcn_readfirstlane(all ? c : s_list[c]);
        const rbsm_prim &q = prims[k];
        const float z = q.depth;
        for (int e = 0; e < 4; ++e)
            if (col + e <= i1 && z < d[e] && covers(q, px[e], py)) d[e] = z;
    }
    float *dst = map + (int64_t)row * pitch + col;
    for (int e = 0; e < 4; ++e)
        if (col + e <= i1) dst[e] = d[e];
}

inline void launch_raster(const rbsm_prim *prims, int n, double r0, double ru, double rv, int W, int H, int64_t pitch,
                          float *map, hipStream_t stream) {
    const int tiles_x = (W + kRasTile - 1) / kRasTile, tiles_y = (H + kRasTile - 1) / kRasTile;
    hipLaunchKernelGGL(raster_kernel, dim3((unsigned)((int64_t)tiles_x * tiles_y)), dim3(kRasT), 0, stream, prims, n,
                       r0, ru, rv, W, H, pitch, map, tiles_x);
}

}  // namespace rbsm
