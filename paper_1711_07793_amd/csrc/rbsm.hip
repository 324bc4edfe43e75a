// RBSM / RSMSS per-fragment shadow pass for MI355X (gfx950) and its C ABI.
//
// Kernels: one lane per fragment, fragments streamed in input order (so a
// wave reads 768 contiguous bytes of (u, v, z) and writes 64 contiguous
// outputs), shadow-map reads through the vector L1/L2.  See rbsm.h for the
// contract of each entry point.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "rbsm.h"
#include "rbsm_device.hpp"

using namespace rbsm;

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void sm_kernel(MapView m, const float *__restrict__ frags,
                                                    int64_t n, float bias, uint8_t *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const float u = frags[3 * k + 0], v = frags[3 * k + 1], z = frags[3 * k + 2];
    const Addr a = address(u, v, z, m.W, m.H, bias);
    out[k] = lit(a.zb, texel(m, a.i0, a.j0)) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void hard_kernel(MapView m, const float *__restrict__ frags,
                                                      int64_t n, float bias, int maxd,
                                                      uint8_t *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const float u = frags[3 * k + 0], v = frags[3 * k + 1], z = frags[3 * k + 2];
    const Addr a = address(u, v, z, m.W, m.H, bias);
    out[k] = eval_texel<true>(m, a.i0, a.j0, a.fx, a.fy, a.zb, maxd) != 0.0f ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void rsmss_kernel(MapView m, const float *__restrict__ frags,
                                                       int64_t n, float bias, int maxd,
                                                       float *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const float u = frags[3 * k + 0], v = frags[3 * k + 1], z = frags[3 * k + 2];
    const Addr a = address(u, v, z, m.W, m.H, bias);
    out[k] = eval_texel<false>(m, a.i0, a.j0, a.fx, a.fy, a.zb, maxd);
}

// RPCF: box average of RSMSS over the (2r+1)^2 texel offsets, a-major.
__global__ __launch_bounds__(kBlock) void rpcf_kernel(MapView m, const float *__restrict__ frags,
                                                      int64_t n, float bias, int maxd, int r,
                                                      float inv_count, float *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const float u = frags[3 * k + 0], v = frags[3 * k + 1], z = frags[3 * k + 2];
    const Addr a = address(u, v, z, m.W, m.H, bias);
    float sum = 0.0f;
    for (int da = -r; da <= r; ++da)
        for (int db = -r; db <= r; ++db)
            sum += eval_texel<false>(m, a.i0 + da, a.j0 + db, a.fx, a.fy, a.zb, maxd);
    out[k] = sum * inv_count;
}

// Read-set marking (instrumentation).  Mirrors the reads of the paper's
// listings: computeN at every traversal texel that keeps the test result.
struct Marker {
    MapView m;
    uint8_t *touched;
    __device__ __forceinline__ float read(int i, int j) const {
        i = min(max(i, 0), m.W - 1);
        j = min(max(j, 0), m.H - 1);
        touched[(int64_t)j * m.W + i] = 1;
        return m.t[(int64_t)j * m.pitch + i];
    }
    __device__ __forceinline__ unsigned mask(int i, int j, float zb, bool s) const {
        unsigned b = 0;
        b |= (lit(zb, read(i - 1, j)) != s) ? BIT_L : 0u;
        b |= (lit(zb, read(i + 1, j)) != s) ? BIT_R : 0u;
        b |= (lit(zb, read(i, j + 1)) != s) ? BIT_T : 0u;
        b |= (lit(zb, read(i, j - 1)) != s) ? BIT_B : 0u;
        return b;
    }
    __device__ void walk(int i, int j, int dx, int dy, float zb, bool s, unsigned m0, int maxd) const {
        for (int k = 1; k <= maxd; ++k) {
            i += dx;
            j += dy;
            if (lit(zb, read(i, j)) != s) return;
            if ((mask(i, j, zb, s) & m0) == 0u) return;
        }
    }
    __device__ void texel_reads(int i0, int j0, float zb, int maxd, bool hard) const {
        const bool s = lit(zb, read(i0, j0));
        if (hard && !s) return;
        const unsigned m0 = mask(i0, j0, zb, s);
        if (m0 == 0u) return;
        walk(i0, j0, -1, 0, zb, s, m0, maxd);
        walk(i0, j0, +1, 0, zb, s, m0, maxd);
        walk(i0, j0, 0, +1, zb, s, m0, maxd);
        walk(i0, j0, 0, -1, zb, s, m0, maxd);
    }
};

__global__ __launch_bounds__(kBlock) void footprint_kernel(Marker mk, const float *__restrict__ frags,
                                                           int64_t n, float bias, int maxd, int r,
                                                           int hard) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const float u = frags[3 * k + 0], v = frags[3 * k + 1], z = frags[3 * k + 2];
    const Addr a = address(u, v, z, mk.m.W, mk.m.H, bias);
    for (int da = -r; da <= r; ++da)
        for (int db = -r; db <= r; ++db) mk.texel_reads(a.i0 + da, a.j0 + db, a.zb, maxd, hard != 0);
}

// ---------------------------------------------------------------------------
// host side: validation and launch
// ---------------------------------------------------------------------------

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, const char *detail = nullptr) {
    snprintf(g_err, sizeof(g_err), fmt, detail ? detail : "");
    return code;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

// Common checks; on success fills the map view.
int validate(const char *fn, const float *map, const float *frags, int64_t n, const rbsm_params *p,
             const void *out, size_t out_elem, bool allow_radius, MapView *mv) {
    if (!p) return fail(RBSM_ERR_INVALID_ARG, "%s: params is null", fn);
    if (p->width < 1 || p->height < 1 || p->width > 65536 || p->height > 65536)
        return fail(RBSM_ERR_INVALID_ARG, "%s: width and height must be in 1..65536", fn);
    if (p->pitch < p->width) return fail(RBSM_ERR_INVALID_ARG, "%s: pitch < width", fn);
    if (p->max_dist < 1 || p->max_dist > 64)
        return fail(RBSM_ERR_INVALID_ARG, "%s: max_dist must be in 1..64", fn);
    if (p->kernel_radius < 0 || p->kernel_radius > 32)
        return fail(RBSM_ERR_INVALID_ARG, "%s: kernel_radius must be in 0..32", fn);
    if (!allow_radius && p->kernel_radius != 0)
        return fail(RBSM_ERR_INVALID_ARG, "%s: kernel_radius must be 0 for this entry point", fn);
    if (n < 0) return fail(RBSM_ERR_INVALID_ARG, "%s: n < 0", fn);
    if (n > ((int64_t)1 << 40)) return fail(RBSM_ERR_INVALID_ARG, "%s: n too large", fn);
    if (n > 0) {
        if (!map || !frags || !out) return fail(RBSM_ERR_INVALID_ARG, "%s: null array pointer", fn);
        const size_t map_bytes = ((size_t)(p->height - 1) * (size_t)p->pitch + (size_t)p->width) * 4u;
        const size_t out_bytes = (size_t)n * out_elem;
        if (overlaps(out, out_bytes, map, map_bytes) || overlaps(out, out_bytes, frags, (size_t)n * 12u))
            return fail(RBSM_ERR_INVALID_ARG, "%s: output overlaps an input", fn);
    }
    mv->t = map;
    mv->pitch = p->pitch;
    mv->W = p->width;
    mv->H = p->height;
    return RBSM_OK;
}

int launched(const char *fn) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        snprintf(g_err, sizeof(g_err), "%s: launch failed: %s", fn, hipGetErrorString(e));
        return RBSM_ERR_HIP;
    }
    return RBSM_OK;
}

unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

extern "C" {

int rbsm_visibility(const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                    uint8_t *out_mask, hipStream_t stream) {
    MapView mv;
    const int st = validate("rbsm_visibility", shadow_map, frags, n, p, out_mask, 1, false, &mv);
    if (st != RBSM_OK) return st;
    if (n == 0) return RBSM_OK;
    hipLaunchKernelGGL(hard_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, mv, frags, n,
                       p->depth_bias, p->max_dist, out_mask);
    return launched("rbsm_visibility");
}

int rsmss_visibility(const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                     float *out_vis, hipStream_t stream) {
    MapView mv;
    const int st = validate("rsmss_visibility", shadow_map, frags, n, p, out_vis, 4, true, &mv);
    if (st != RBSM_OK) return st;
    if (n == 0) return RBSM_OK;
    const int r = p->kernel_radius;
    if (r == 0) {
        hipLaunchKernelGGL(rsmss_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, mv, frags, n,
                           p->depth_bias, p->max_dist, out_vis);
    } else {
        const float inv = 1.0f / (float)((2 * r + 1) * (2 * r + 1));
        hipLaunchKernelGGL(rpcf_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, mv, frags, n,
                           p->depth_bias, p->max_dist, r, inv, out_vis);
    }
    return launched("rsmss_visibility");
}

int sm_visibility(const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                  uint8_t *out_mask, hipStream_t stream) {
    MapView mv;
    rbsm_params q = p ? *p : rbsm_params{};
    if (p) {
        q.max_dist = 1;
        q.kernel_radius = 0;
    }
    const int st = validate("sm_visibility", shadow_map, frags, n, p ? &q : nullptr, out_mask, 1, false, &mv);
    if (st != RBSM_OK) return st;
    if (n == 0) return RBSM_OK;
    hipLaunchKernelGGL(sm_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, mv, frags, n,
                       p->depth_bias, out_mask);
    return launched("sm_visibility");
}

int rbsm_footprint(const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                   int32_t mode, uint8_t *touched, hipStream_t stream) {
    if (mode != 0 && mode != 1) return fail(RBSM_ERR_INVALID_ARG, "rbsm_footprint: mode must be 0 or 1");
    MapView mv;
    const int st = validate("rbsm_footprint", shadow_map, frags, n, p, touched, 0, mode == 1, &mv);
    if (st != RBSM_OK) return st;
    if (n == 0) return RBSM_OK;
    if (!touched) return fail(RBSM_ERR_INVALID_ARG, "rbsm_footprint: touched is null");
    const size_t tb = (size_t)p->width * (size_t)p->height;
    const size_t map_bytes = ((size_t)(p->height - 1) * (size_t)p->pitch + (size_t)p->width) * 4u;
    if (overlaps(touched, tb, shadow_map, map_bytes) || overlaps(touched, tb, frags, (size_t)n * 12u))
        return fail(RBSM_ERR_INVALID_ARG, "rbsm_footprint: touched overlaps an input");
    Marker mk{mv, touched};
    hipLaunchKernelGGL(footprint_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, mk, frags, n,
                       p->depth_bias, p->max_dist, mode == 1 ? p->kernel_radius : 0, mode == 0 ? 1 : 0);
    return launched("rbsm_footprint");
}

const char *rbsm_last_error(void) { return g_err; }

int32_t rbsm_abi_version(void) { return 100; }

}  // extern "C"
