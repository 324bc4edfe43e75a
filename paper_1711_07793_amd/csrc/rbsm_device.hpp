// Device-side building blocks of the RBSM / RSMSS per-fragment pass for gfx950.
//
// Every function here works on one texel neighbourhood of one fragment; the
// kernels decide how fragments map to lanes.  Arithmetic is binary32 in the
// order of the paper's listings, compiled without FMA contraction, so results
// are bit-reproducible against any IEEE binary32 evaluation in that order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbsm {

// Discontinuity bits of a texel: its left / right / top (+y) / bottom (-y)
// neighbour has the opposite shadow test result (Eq. 3).
enum : unsigned { BIT_L = 1u, BIT_R = 2u, BIT_T = 4u, BIT_B = 8u };

struct MapView {
    const float *__restrict__ t;
    int64_t pitch;
    int W, H;
};

// Loads and stores of device buffers through global-address-space pointers:
// pointers read from a job table in memory are otherwise generic, and the
// compiler then emits flat instructions, which count against the LDS counter
// too, so every LDS wait also waits for memory (and back-to-back loads of one
// fragment were serialised).
template <class T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ void gst(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}
// 12-byte loads (three consecutive texels, 4-byte aligned) through a native
// vector type whose alignment is lowered to 4, so the load is exactly 12 bytes.
typedef float f32x3 __attribute__((ext_vector_type(3), aligned(4)));
__device__ __forceinline__ f32x3 gld3(const float *p) {
    return *(const __attribute__((address_space(1))) f32x3 *)p;
}
// 16-byte load of four consecutive texels at 4-byte alignment (map rows).
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ f32x4u gld4u(const float *p) {
    return *(const __attribute__((address_space(1))) f32x4u *)p;
}
// 16-byte forms through a native vector type (HIP's float4 is a class whose
// copy takes a generic reference, which would bring the flat access back).
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 gld4(const float4 *p) {
    const f32x4 v = *(const __attribute__((address_space(1))) f32x4 *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gst4(float4 *p, float4 v) {
    f32x4 w;
    w.x = v.x; w.y = v.y; w.z = v.z; w.w = v.w;
    *(__attribute__((address_space(1))) f32x4 *)p = w;
}

// Nearest-texel fetch with clamp-to-edge.
__device__ __forceinline__ float texel(const MapView &m, int i, int j) {
    i = min(max(i, 0), m.W - 1);
    j = min(max(j, 0), m.H - 1);
    return gld(m.t + ((int64_t)j * m.pitch + i));
}

// Eq. 1: lit (1) unless the biased fragment depth lies behind the blocker.
__device__ __forceinline__ bool lit(float zb, float t) { return !(zb > t); }

struct Addr {
    int i0, j0;   // texel of the fragment
    float fx, fy; // sub-texel position in [0, 1)
    float zb;     // z - bias
};

// Texel and sub-texel position of a light-space fragment.  The integer index
// is clamped to +-2^20, which cannot change any read on maps of at most 2^16
// texels per side with reach below 2^10.
__device__ __forceinline__ Addr address(float u, float v, float z, int W, int H, float bias) {
    Addr a;
    const float X = u * (float)W;
    const float Y = v * (float)H;
    const float flx = floorf(X), fly = floorf(Y);
    a.fx = X - flx;
    a.fy = Y - fly;
    a.i0 = (int)fminf(fmaxf(flx, -1048576.0f), 1048576.0f);
    a.j0 = (int)fminf(fmaxf(fly, -1048576.0f), 1048576.0f);
    a.zb = z - bias;
    return a;
}

// Bounded traversal along (DX, DY) (Listing 3 with the shared-direction test
// of Sec. 3.1.3).  Returns +k when the k-th texel has the opposite test (an
// edge end), -k when the k-th texel stops sharing a discontinuity direction
// with the fragment, -(maxd + 1) when the walk runs out.
//
// Only discontinuity bits perpendicular to the walk can be shared: the texel
// behind a visited texel has the fragment's test result, and a fragment with a
// discontinuity in the walking direction ends its walk at k = 1.  So a step
// reads the visited texel and at most its two perpendicular neighbours, and
// only those whose bit is set in the fragment's mask m0.
template <int DX, int DY>
__device__ __forceinline__ int walk(const MapView &m, int i0, int j0, float zb, bool s, unsigned m0,
                                    int maxd) {
    const bool chk_a = DX != 0 ? (m0 & BIT_T) != 0 : (m0 & BIT_L) != 0;
    const bool chk_b = DX != 0 ? (m0 & BIT_B) != 0 : (m0 & BIT_R) != 0;
    int i = i0, j = j0;
    for (int k = 1; k <= maxd; ++k) {
        i += DX;
        j += DY;
        if (lit(zb, texel(m, i, j)) != s) return k;
        bool share = false;
        if (chk_a) share |= lit(zb, DX != 0 ? texel(m, i, j + 1) : texel(m, i - 1, j)) != s;
        if (chk_b) share |= lit(zb, DX != 0 ? texel(m, i, j - 1) : texel(m, i + 1, j)) != s;
        if (!share) return -k;
    }
    return -(maxd + 1);
}

// The same traversal with the direction as a run-time value, so lanes that
// walk different directions of different fragments share one instruction
// stream.  (dx, dy) is one of (-1,0), (1,0), (0,1), (0,-1).
__device__ __forceinline__ int walk_dir(const MapView &m, int i0, int j0, float zb, bool s, unsigned m0,
                                        int maxd, int dx, int dy) {
    const bool horiz = dx != 0;
    const bool chk_a = horiz ? (m0 & BIT_T) != 0 : (m0 & BIT_L) != 0;
    const bool chk_b = horiz ? (m0 & BIT_B) != 0 : (m0 & BIT_R) != 0;
    // offsets of the two perpendicular neighbours: top/bottom or left/right
    const int ax = horiz ? 0 : -1, ay = horiz ? 1 : 0;
    const int bx = horiz ? 0 : 1, by = horiz ? -1 : 0;
    int i = i0, j = j0;
    for (int k = 1; k <= maxd; ++k) {
        i += dx;
        j += dy;
        const float tc = texel(m, i, j);
        const float ta = texel(m, i + ax, j + ay);
        const float tb = texel(m, i + bx, j + by);
        if (lit(zb, tc) != s) return k;
        const bool share = (chk_a && lit(zb, ta) != s) || (chk_b && lit(zb, tb) != s);
        if (!share) return -k;
    }
    return -(maxd + 1);
}

// One axis of the normalized discontinuity space (Eq. 5): the code counts the
// walks that found an end (2 -> 1, 1 -> 0, 0 -> -1); with exactly one end the
// coordinate is the fragment's distance to the end texel's boundary over the
// number of edge texels on the axis; 1 with no end, 0 with two.
struct Axis {
    float nrd;
    int code;
};

__device__ __forceinline__ Axis normalize_axis(int rn, int rp, float f) {
    const int ends = (rn > 0) + (rp > 0);
    const int an = abs(rn), ap = abs(rp);
    const float len = (float)(an + ap - 1);
    const float a = rp > 0 ? (float)rp - f : (float)(an - 1) + f;
    const float q = a / len;
    Axis r;
    r.code = ends == 2 ? 1 : (ends == 0 ? -1 : 0);
    r.nrd = ends == 1 ? q : (ends == 0 ? 1.0f : 0.0f);
    return r;
}

// Listing 4 without shape branches: U/O (code 1 on either axis, which the
// short-U/O test d == 0.75 implies) shadow, and with nrd = 1 on an axis
// without ends the I shape falls out of the L-line test.
__device__ __forceinline__ float vis_hard(Axis x, Axis y) {
    const bool keep = (x.code != 1) & (y.code != 1) & !(y.nrd < 1.0f - x.nrd);
    return keep ? 1.0f : 0.0f;
}

// Listing 5 without shape branches: code-1 axes contribute 0 (O flips the
// test, U ramps along the other axis), an axis without ends contributes 1
// (the I shape returns the test), and the rest is the L ramp
// clamp((d.z + sign*ty) + sign*tx, 0, 1) with sign = 1 - 2 d.z.
__device__ __forceinline__ float vis_rsmss(bool s, Axis x, Axis y) {
    const float tx = x.code == 1 ? 0.0f : x.nrd;
    const float ty = y.code == 1 ? 0.0f : y.nrd;
    const float v = s ? (ty + tx) : ((1.0f - ty) - tx);
    const float lo = v > 0.0f ? v : 0.0f;
    return lo < 1.0f ? lo : 1.0f;
}

// Discontinuity mask of texel (i, j) at depth zb, given its own test s.
__device__ __forceinline__ unsigned mask_of(const MapView &m, int i, int j, float zb, bool s) {
    unsigned b = 0;
    b |= (lit(zb, texel(m, i - 1, j)) != s) ? BIT_L : 0u;
    b |= (lit(zb, texel(m, i + 1, j)) != s) ? BIT_R : 0u;
    b |= (lit(zb, texel(m, i, j + 1)) != s) ? BIT_T : 0u;
    b |= (lit(zb, texel(m, i, j - 1)) != s) ? BIT_B : 0u;
    return b;
}

// Visibility of a fragment whose texel is (i0, j0): Listing 1 with the
// hard (HARD) or filtering visibility function.
template <bool HARD>
__device__ __forceinline__ float eval_texel(const MapView &m, int i0, int j0, float fx, float fy,
                                            float zb, int maxd) {
    const bool s = lit(zb, texel(m, i0, j0));
    if (HARD && !s) return 0.0f;
    const unsigned m0 = mask_of(m, i0, j0, zb, s);
    if (m0 == 0u) return s ? 1.0f : 0.0f;
    const int rl = walk<-1, 0>(m, i0, j0, zb, s, m0, maxd);
    const int rr = walk<+1, 0>(m, i0, j0, zb, s, m0, maxd);
    const int rt = walk<0, +1>(m, i0, j0, zb, s, m0, maxd);
    const int rb = walk<0, -1>(m, i0, j0, zb, s, m0, maxd);
    const Axis ax = normalize_axis(rl, rr, fx);
    const Axis ay = normalize_axis(rb, rt, fy);
    return HARD ? vis_hard(ax, ay) : vis_rsmss(s, ax, ay);
}

}  // namespace rbsm
