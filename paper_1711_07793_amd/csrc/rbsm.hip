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

#include <algorithm>
#include <new>
#include <vector>

#include <algorithm>

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

// XCD-aware block order.  Workgroups are handed to the 8 XCDs round-robin;
// renumber them so each XCD (and its private L2) works through one
// contiguous range of fragments.  A bijection for any grid size.
__device__ __forceinline__ int64_t xcd_block(int b, int nb) {
    const int x = b & 7, local = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return x < rem ? (int64_t)x * (per + 1) + local
                   : (int64_t)rem * (per + 1) + (int64_t)(x - rem) * per + local;
}

// ---------------------------------------------------------------------------
// Main pass: 2-D screen tiles with their light-space footprint staged in LDS.
// ---------------------------------------------------------------------------

constexpr int kT = 256;            // threads per workgroup
constexpr int kF = 4;              // consecutive pixels per thread
constexpr int kTileF = kT * kF;    // fragments per tile
constexpr int kState = 256;        // edge fragments whose full state is kept in LDS
constexpr int kLdsSteps = 8;       // traversal steps per block, all reads issued together

// Staged light-space footprint of one screen tile: texels [by0..by1] x
// [bx0..bx1] of the map (clamped coordinates), row-major with stride bw.
struct Staged {
    const float *lds;
    int bx0, by0, bx1, by1, bw;
    bool on;
};

__device__ __forceinline__ int clampi(int x, int n) { return min(max(x, 0), n - 1); }

// Copy texels [y0, y0+h) x [x0, x0+w) of the map into dst (row-major, stride
// w), the workgroup's kT threads striding over the rectangle.
__device__ __forceinline__ void stage_rect(const MapView &m, float *dst, int x0, int y0, int w, int h, int t) {
    const int area = w * h;
    int r = t / w, c = t % w;
    const int dr = kT / w, dc = kT % w;
    for (int idx = t; idx < area; idx += kT) {
        dst[idx] = m.t[(int64_t)(y0 + r) * m.pitch + (x0 + c)];
        r += dr;
        c += dc;
        if (c >= w) {
            c -= w;
            ++r;
        }
    }
}

// Is texel (i, j), clamped, in the staged box?  Returns its LDS index or -1.
__device__ __forceinline__ int staged_index(const MapView &m, const Staged &st, int i, int j) {
    i = min(max(i, 0), m.W - 1);
    j = min(max(j, 0), m.H - 1);
    if (!st.on || i < st.bx0 || i > st.bx1 || j < st.by0 || j > st.by1) return -1;
    return (j - st.by0) * st.bw + (i - st.bx0);
}

// Clamp-to-edge read: LDS inside the staged box, global memory outside.
__device__ __forceinline__ float fetch(const MapView &m, const Staged &st, int i, int j) {
    const int li = staged_index(m, st, i, j);
    if (li >= 0) return st.lds[li];
    i = min(max(i, 0), m.W - 1);
    j = min(max(j, 0), m.H - 1);
    return m.t[(int64_t)j * m.pitch + i];
}

// One workgroup owns a TW x (1024/TW) pixel tile of a row-major image of
// width vw (flat mode: vw = n, TW = 1024); each thread owns 4 consecutive
// pixels of one row (one 48-byte fragment load, one packed store).
//  1. load fragments; the workgroup reduces the bounding box of their texels,
//     grows it by `apron` texels and, when it holds at most `cap` texels,
//     copies it into LDS with row-contiguous loads (else reads stay global);
//  2. centre and neighbour tests; fragments without a discontinuity (and, in
//     hard mode, shadowed ones) are final and stored at once;
//  3. edge fragments are compacted with wave ballots into an LDS queue that
//     keeps their texel, depth, sub-texel position, test and mask;
//  4. tiles with edge fragments restage: a horizontal band (the box rows
//     +-1, columns +-(MAXDIST+1)) and a vertical band (the box columns +-1,
//     rows +-(MAXDIST+1)) hold every texel any traversal of the tile reads;
//  5. one lane per (edge fragment, direction) walks in blocks of 8 steps,
//     all reads of a block issued together, from the bands (from global
//     memory when the bands exceed the LDS capacity);
//  6. one lane per edge fragment normalizes, evaluates the visibility
//     function and stores.
// Staging, tile shape and queues only decide where texels are read from and
// by which lane: every result equals the per-fragment listing.
// Workgroup-shared state of one tile (the staged texels live in the dynamic
// LDS array that follows it).
struct TileShared {
    int box[kT / 64][4];
    int16_t slot[kTileF];
    uint8_t sm[kTileF];    // bit 4: centre test, bits 0-3: discontinuity mask
    int qi[kState], qj[kState];
    float qz[kState], qfx[kState], qfy[kState];
    int8_t rd[kTileF][4];  // left, right, top, bottom
    int count;
};

template <bool HARD, int TW>
__device__ __forceinline__ void process_tile(MapView m, const float *__restrict__ frags, int64_t n, int64_t vw,
                                             int64_t tiles_x, float bias, int maxd, int apron, int cap,
                                             int vec_ok, void *__restrict__ out_v, int64_t tile_id,
                                             TileShared &sh, float *s_tex) {
    constexpr int TH = kTileF / TW;
    constexpr int LPR = TW / kF;
    auto &s_box = sh.box;
    auto &q_slot = sh.slot;
    auto &q_sm = sh.sm;
    auto &q_i = sh.qi;
    auto &q_j = sh.qj;
    auto &q_z = sh.qz;
    auto &q_fx = sh.qfx;
    auto &q_fy = sh.qfy;
    auto &q_rd = sh.rd;
    int &q_count = sh.count;

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int64_t tyi = tile_id / tiles_x, txi = tile_id % tiles_x;
    const int64_t px0 = txi * TW + (int64_t)(t % LPR) * kF;
    const int64_t k0 = (tyi * TH + t / LPR) * vw + px0;
    const unsigned long long below = __lanemask_lt();

    Staged st;
    int core_i0, core_i1, core_j0, core_j1;  // clamped texel box of the tile's fragments
    {
        bool valid[kF];
#pragma unroll
        for (int f = 0; f < kF; ++f) valid[f] = (px0 + f < vw) && (k0 + f < n);
        const bool full = vec_ok && valid[kF - 1];

        float fr[3 * kF];
        if (full) {
            const float4 *p4 = reinterpret_cast<const float4 *>(frags + 3 * k0);
            const float4 a = p4[0], b = p4[1], c = p4[2];
            fr[0] = a.x; fr[1] = a.y; fr[2] = a.z; fr[3] = a.w;
            fr[4] = b.x; fr[5] = b.y; fr[6] = b.z; fr[7] = b.w;
            fr[8] = c.x; fr[9] = c.y; fr[10] = c.z; fr[11] = c.w;
        } else {
#pragma unroll
            for (int f = 0; f < kF; ++f) {
                const int64_t k = k0 + f;
                fr[3 * f + 0] = valid[f] ? frags[3 * k + 0] : 0.0f;
                fr[3 * f + 1] = valid[f] ? frags[3 * k + 1] : 0.0f;
                fr[3 * f + 2] = valid[f] ? frags[3 * k + 2] : 0.0f;
            }
        }

        Addr ad[kF];
        int imin = INT32_MAX, imax = INT32_MIN, jmin = INT32_MAX, jmax = INT32_MIN;
#pragma unroll
        for (int f = 0; f < kF; ++f) {
            ad[f] = address(fr[3 * f], fr[3 * f + 1], fr[3 * f + 2], m.W, m.H, bias);
            if (valid[f]) {
                const int ic = min(max(ad[f].i0, 0), m.W - 1), jc = min(max(ad[f].j0, 0), m.H - 1);
                imin = min(imin, ic); imax = max(imax, ic);
                jmin = min(jmin, jc); jmax = max(jmax, jc);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            imin = min(imin, __shfl_xor(imin, off));
            imax = max(imax, __shfl_xor(imax, off));
            jmin = min(jmin, __shfl_xor(jmin, off));
            jmax = max(jmax, __shfl_xor(jmax, off));
        }
        if (lane == 0) {
            s_box[wave][0] = imin; s_box[wave][1] = imax;
            s_box[wave][2] = jmin; s_box[wave][3] = jmax;
        }
        if (t == 0) q_count = 0;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kT / 64; ++w) {
            imin = min(imin, s_box[w][0]); imax = max(imax, s_box[w][1]);
            jmin = min(jmin, s_box[w][2]); jmax = max(jmax, s_box[w][3]);
        }
        core_i0 = imin; core_i1 = imax; core_j0 = jmin; core_j1 = jmax;
        st.lds = s_tex;
        st.bx0 = max(imin - apron, 0);
        st.bx1 = min(imax + apron, m.W - 1);
        st.by0 = max(jmin - apron, 0);
        st.by1 = min(jmax + apron, m.H - 1);
        st.bw = st.bx1 - st.bx0 + 1;
        const int bh = st.by1 - st.by0 + 1;
        st.on = imin <= imax && (int64_t)st.bw * bh <= (int64_t)cap;
        if (st.on) stage_rect(m, s_tex, st.bx0, st.by0, st.bw, bh, t);
        __syncthreads();

        bool s[kF], edge[kF];
        unsigned m0[kF];
#pragma unroll
        for (int f = 0; f < kF; ++f) {
            float cl = 0.0f, cc = 0.0f, cr = 0.0f, ct = 0.0f, cb = 0.0f;
            if (valid[f]) {
                const int ti = min(max(ad[f].i0, 0), m.W - 1), tj = min(max(ad[f].j0, 0), m.H - 1);
                const int il = max(ti - 1, 0), ir = min(ti + 1, m.W - 1);
                const int jl = max(tj - 1, 0), jh = min(tj + 1, m.H - 1);
                if (st.on) {
                    const int rc = (tj - st.by0) * st.bw - st.bx0;
                    cl = s_tex[rc + il];
                    cc = s_tex[rc + ti];
                    cr = s_tex[rc + ir];
                    ct = s_tex[(jh - st.by0) * st.bw - st.bx0 + ti];
                    cb = s_tex[(jl - st.by0) * st.bw - st.bx0 + ti];
                } else {
                    const float *row = m.t + (int64_t)tj * m.pitch;
                    cl = row[il];
                    cc = row[ti];
                    cr = row[ir];
                    ct = m.t[(int64_t)jh * m.pitch + ti];
                    cb = m.t[(int64_t)jl * m.pitch + ti];
                }
            }
            const float zb = ad[f].zb;
            s[f] = lit(zb, cc);
            m0[f] = ((lit(zb, cl) != s[f]) ? BIT_L : 0u) | ((lit(zb, cr) != s[f]) ? BIT_R : 0u) |
                    ((lit(zb, ct) != s[f]) ? BIT_T : 0u) | ((lit(zb, cb) != s[f]) ? BIT_B : 0u);
            edge[f] = valid[f] && m0[f] != 0u && (!HARD || s[f]);
        }

        // final results of every fragment that is not an edge fragment
        const bool any_edge = edge[0] | edge[1] | edge[2] | edge[3];
        if (HARD) {
            uint8_t *out = static_cast<uint8_t *>(out_v);
            if (full && !any_edge) {
                uint32_t packed = 0;
#pragma unroll
                for (int f = 0; f < kF; ++f) packed |= (uint32_t)(s[f] ? 1u : 0u) << (8 * f);
                *reinterpret_cast<uint32_t *>(out + k0) = packed;
            } else {
#pragma unroll
                for (int f = 0; f < kF; ++f)
                    if (valid[f] && !edge[f]) out[k0 + f] = s[f] ? 1 : 0;
            }
        } else {
            float *out = static_cast<float *>(out_v);
            if (full && !any_edge) {
                *reinterpret_cast<float4 *>(out + k0) =
                    make_float4(s[0] ? 1.0f : 0.0f, s[1] ? 1.0f : 0.0f, s[2] ? 1.0f : 0.0f, s[3] ? 1.0f : 0.0f);
            } else {
#pragma unroll
                for (int f = 0; f < kF; ++f)
                    if (valid[f] && !edge[f]) out[k0 + f] = s[f] ? 1.0f : 0.0f;
            }
        }

        // queue the edge fragments: wave ballots, one LDS atomic per wave
        unsigned long long bal[kF];
        int wave_total = 0;
#pragma unroll
        for (int f = 0; f < kF; ++f) {
            bal[f] = __ballot(edge[f]);
            wave_total += __popcll(bal[f]);
        }
        if (wave_total) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&q_count, wave_total);
            base = __shfl(base, 0);
#pragma unroll
            for (int f = 0; f < kF; ++f) {
                const int pos = base + __popcll(bal[f] & below);
                if (edge[f]) {
                    q_slot[pos] = (int16_t)(kF * t + f);
                    q_sm[pos] = (uint8_t)(m0[f] | (s[f] ? 16u : 0u));
                    if (pos < kState) {
                        q_i[pos] = ad[f].i0;
                        q_j[pos] = ad[f].j0;
                        q_z[pos] = ad[f].zb;
                        q_fx[pos] = ad[f].fx;
                        q_fy[pos] = ad[f].fy;
                    }
                }
                base += __popcll(bal[f]);
            }
        }
    }
    __syncthreads();
    const int ne = q_count;
    if (ne == 0) return;

    // fragment index of queue entry e
    auto frag_of = [&](int e) -> int64_t {
        const int slot = q_slot[e];
        const int owner = slot >> 2, f = slot & 3;
        return (tyi * TH + owner / LPR) * vw + txi * TW + (int64_t)(owner % LPR) * kF + f;
    };
    // full state of queue entry e (from LDS, or recomputed past kState)
    auto state_of = [&](int e, int &i0, int &j0, float &zb, float &fx, float &fy) {
        if (e < kState) {
            i0 = q_i[e]; j0 = q_j[e]; zb = q_z[e]; fx = q_fx[e]; fy = q_fy[e];
        } else {
            const int64_t k = frag_of(e);
            const Addr b = address(frags[3 * k], frags[3 * k + 1], frags[3 * k + 2], m.W, m.H, bias);
            i0 = b.i0; j0 = b.j0; zb = b.zb; fx = b.fx; fy = b.fy;
        }
    };

    // 4. restage: every texel a traversal of this tile can read lies in a
    //    horizontal band (the core rows +-1, the core columns +-(maxd+1)) or
    //    a vertical band (the core columns +-1, the core rows +-(maxd+1));
    //    copy both into LDS over the core box when they fit
    const int reach = maxd + 1;
    const int hx0 = max(core_i0 - reach, 0), hx1 = min(core_i1 + reach, m.W - 1);
    const int hy0 = max(core_j0 - 1, 0), hy1 = min(core_j1 + 1, m.H - 1);
    const int vx0 = max(core_i0 - 1, 0), vx1 = min(core_i1 + 1, m.W - 1);
    const int vy0 = max(core_j0 - reach, 0), vy1 = min(core_j1 + reach, m.H - 1);
    const int hw = hx1 - hx0 + 1, hh = hy1 - hy0 + 1;
    const int vwid = vx1 - vx0 + 1, vh = vy1 - vy0 + 1;
    // both bands at once when they fit together, else one after the other
    const bool both = (int64_t)hw * hh + (int64_t)vwid * vh <= (int64_t)cap;
    const bool h_fits = (int64_t)hw * hh <= (int64_t)cap, v_fits = (int64_t)vwid * vh <= (int64_t)cap;
    for (int pass = 0; pass < (both ? 1 : 2); ++pass) {
        // pass covers directions [d_lo, d_hi): 0 left, 1 right, 2 top, 3 bottom
        const int d_lo = both ? 0 : 2 * pass, d_hi = both ? 4 : 2 * pass + 2;
        const bool h_on = both || (pass == 0 && h_fits);
        const bool v_on = both || (pass == 1 && v_fits);
        float *s_h = s_tex, *s_v = both ? s_tex + hw * hh : s_tex;
        if (pass == 1) __syncthreads();  // pass 0 walks are done with s_tex
        if (h_on && d_lo == 0) stage_rect(m, s_h, hx0, hy0, hw, hh, t);
        if (v_on && d_hi == 4) stage_rect(m, s_v, vx0, vy0, vwid, vh, t);
        __syncthreads();

        // 5. walks, one lane per (fragment, direction), blocks of kLdsSteps
        //    steps with all reads of a block issued together (global memory
        //    when the band did not fit)
        const int nd = d_hi - d_lo;
        for (int task = t; task < nd * ne; task += kT) {
            const int e = task / nd, dir = d_lo + task % nd;
            int i0, j0;
            float zb, fx, fy;
            state_of(e, i0, j0, zb, fx, fy);
            const unsigned sm = q_sm[e];
            const bool s = (sm & 16u) != 0;
            const int dx = dir == 0 ? -1 : (dir == 1 ? 1 : 0);
            const int dy = dir == 2 ? 1 : (dir == 3 ? -1 : 0);
            const bool horiz = dx != 0;
            const bool chk_a = horiz ? (sm & BIT_T) != 0 : (sm & BIT_L) != 0;
            const bool chk_b = horiz ? (sm & BIT_B) != 0 : (sm & BIT_R) != 0;
            // band of this walk: rows (or columns) of the fragment +-1
            const bool in_lds = horiz ? h_on : v_on;
            const float *band = horiz ? s_h : s_v;
            const int bx0 = horiz ? hx0 : vx0, by0 = horiz ? hy0 : vy0, bstride = horiz ? hw : vwid;
            const int pa_x = horiz ? 0 : -1, pa_y = horiz ? 1 : 0;
            const int pb_x = horiz ? 0 : 1, pb_y = horiz ? -1 : 0;
            int rd = -(maxd + 1);
            for (int k = 1; k <= maxd; k += kLdsSteps) {
                float tc[kLdsSteps], ta[kLdsSteps], tb[kLdsSteps];
#pragma unroll
                for (int u = 0; u < kLdsSteps; ++u) {
                    const int ku = min(k + u, maxd);
                    const int i = i0 + ku * dx, j = j0 + ku * dy;
                    if (in_lds) {
                        tc[u] = band[(clampi(j, m.H) - by0) * bstride + clampi(i, m.W) - bx0];
                        ta[u] = band[(clampi(j + pa_y, m.H) - by0) * bstride + clampi(i + pa_x, m.W) - bx0];
                        tb[u] = band[(clampi(j + pb_y, m.H) - by0) * bstride + clampi(i + pb_x, m.W) - bx0];
                    } else {
                        tc[u] = texel(m, i, j);
                        ta[u] = texel(m, i + pa_x, j + pa_y);
                        tb[u] = texel(m, i + pb_x, j + pb_y);
                    }
                }
                int stop = 0;
#pragma unroll
                for (int u = kLdsSteps - 1; u >= 0; --u) {
                    const int kk = k + u;
                    if (kk > maxd) continue;
                    const bool end = lit(zb, tc[u]) != s;
                    const bool share = (chk_a && lit(zb, ta[u]) != s) || (chk_b && lit(zb, tb[u]) != s);
                    if (end) stop = kk;
                    else if (!share) stop = -kk;
                }
                if (stop != 0) {
                    rd = stop;
                    break;
                }
            }
            q_rd[e][dir] = (int8_t)rd;
        }
    }
    __syncthreads();

    // 6. normalize, evaluate and store, one lane per edge fragment
    for (int e = t; e < ne; e += kT) {
        int i0, j0;
        float zb, fx, fy;
        state_of(e, i0, j0, zb, fx, fy);
        const bool s = (q_sm[e] & 16u) != 0;
        const Axis axx = normalize_axis(q_rd[e][0], q_rd[e][1], fx);
        const Axis axy = normalize_axis(q_rd[e][3], q_rd[e][2], fy);
        const int64_t k = frag_of(e);
        if (HARD) static_cast<uint8_t *>(out_v)[k] = vis_hard(axx, axy) != 0.0f ? 1 : 0;
        else static_cast<float *>(out_v)[k] = vis_rsmss(s, axx, axy);
    }
}

template <bool HARD, int TW>
__global__ __launch_bounds__(kT) void tile_kernel(MapView m, const float *__restrict__ frags, int64_t n,
                                                  int64_t vw, int64_t tiles_x, float bias, int maxd, int apron,
                                                  int cap, int vec_ok, void *__restrict__ out_v) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    process_tile<HARD, TW>(m, frags, n, vw, tiles_x, bias, maxd, apron, cap, vec_ok, out_v,
                           xcd_block(blockIdx.x, gridDim.x), sh, s_tex);
}

// One job of a batched launch: a (view, light) pass over its own map,
// fragments and output, owning tiles [tile_base, tile_base + tiles).
struct JobDev {
    MapView m;
    const float *frags;
    void *out;
    int64_t n, vw, tiles_x, tile_base;
    float bias;
    int maxd, vec_ok, mode;  // mode 0 hard, 1 RSMSS
};

// Batched pass: one workgroup per tile of any job; block_job maps the
// (XCD-ordered) workgroup index to its job.  Each tile runs exactly the code
// of the single-view pass, so every output is bitwise the same.
template <int TW>
__global__ __launch_bounds__(kT) void batch_kernel(const JobDev *__restrict__ jobs,
                                                   const uint16_t *__restrict__ block_job, int apron, int cap) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    const int64_t g = xcd_block(blockIdx.x, gridDim.x);
    const JobDev J = jobs[block_job[g]];
    const int64_t tile = g - J.tile_base;
    if (J.mode == 0)
        process_tile<true, TW>(J.m, J.frags, J.n, J.vw, J.tiles_x, J.bias, J.maxd, apron, cap, J.vec_ok, J.out,
                               tile, sh, s_tex);
    else
        process_tile<false, TW>(J.m, J.frags, J.n, J.vw, J.tiles_x, J.bias, J.maxd, apron, cap, J.vec_ok, J.out,
                                tile, sh, s_tex);
}

// Launch configuration of the main pass (defaults of the plain entry points).
struct TileConfig {
    int tile_w;   // 16, 32, 64 (2-D tiles) or 1024 (flat)
    int apron;    // texels staged beyond the fragments' texel box, >= 1
    int cap;      // LDS texel capacity per workgroup
};

constexpr TileConfig kDefaultTile{32, 1, 2048};

bool tuning_ok(const rbsm_tuning *t) {
    return t && (t->tile_w == 16 || t->tile_w == 32 || t->tile_w == 64) && t->apron >= 1 && t->apron <= 8 &&
           t->lds_cap >= 256 && t->lds_cap <= 12288;
}

template <bool HARD>
void launch_pass(const MapView &mv, const float *frags, int64_t n, int64_t view_width, float bias, int maxd,
                 TileConfig cfg, void *out, size_t out_align, hipStream_t stream) {
    int64_t vw = view_width;
    int tw = cfg.tile_w;
    if (vw <= 0) {  // flat: one row of n pixels, 1024-fragment chunks
        vw = n;
        tw = 1024;
    }
    const int th = kTileF / tw;
    const int64_t rows = (n + vw - 1) / vw;
    const int64_t tiles_x = (vw + tw - 1) / tw;
    const int64_t tiles = tiles_x * ((rows + th - 1) / th);
    const int vec = ((uintptr_t)frags % 16 == 0) && ((uintptr_t)out % out_align == 0) && (vw % 4 == 0);
    const size_t lds = (size_t)cfg.cap * sizeof(float);
    const dim3 grid((unsigned)tiles), block(kT);
    switch (tw) {
        case 16:
            hipLaunchKernelGGL((tile_kernel<HARD, 16>), grid, block, lds, stream, mv, frags, n, vw, tiles_x, bias,
                               maxd, cfg.apron, cfg.cap, vec, out);
            break;
        case 64:
            hipLaunchKernelGGL((tile_kernel<HARD, 64>), grid, block, lds, stream, mv, frags, n, vw, tiles_x, bias,
                               maxd, cfg.apron, cfg.cap, vec, out);
            break;
        case 1024:
            hipLaunchKernelGGL((tile_kernel<HARD, 1024>), grid, block, lds, stream, mv, frags, n, vw, tiles_x,
                               bias, maxd, cfg.apron, cfg.cap, vec, out);
            break;
        default:
            hipLaunchKernelGGL((tile_kernel<HARD, 32>), grid, block, lds, stream, mv, frags, n, vw, tiles_x, bias,
                               maxd, cfg.apron, cfg.cap, vec, out);
            break;
    }
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
    if (p->view_width < 0) return fail(RBSM_ERR_INVALID_ARG, "%s: view_width < 0", fn);
    if (n > (int64_t)INT32_MAX) return fail(RBSM_ERR_INVALID_ARG, "%s: n exceeds 2^31 - 1", fn);
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

// Tile layout of one job in a batched launch: 2-D tiles of width tw over its
// image (flat jobs are laid out as rows of 1024 fragments).
struct JobLayout {
    int64_t vw, tiles_x, tiles;
};

JobLayout job_layout(int64_t n, int64_t view_width, int tw) {
    JobLayout L;
    L.vw = view_width > 0 ? view_width : 1024;
    const int th = kTileF / tw;
    const int64_t rows = (n + L.vw - 1) / L.vw;
    L.tiles_x = (L.vw + tw - 1) / tw;
    L.tiles = n > 0 ? L.tiles_x * ((rows + th - 1) / th) : 0;
    return L;
}

}  // namespace

struct rbsm_plan {
    int device = 0;
    std::vector<rbsm_job> jobs;
    rbsm_tuning tune{};
    JobDev *d_jobs = nullptr;
    uint16_t *d_block_job = nullptr;
    int64_t blocks = 0;
    int64_t fragments = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void drop_graph(rbsm_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

void free_tables(rbsm_plan *p) {
    if (p->d_jobs) (void)hipFree(p->d_jobs);
    if (p->d_block_job) (void)hipFree(p->d_block_job);
    p->d_jobs = nullptr;
    p->d_block_job = nullptr;
}

// Validate jobs and build (and upload) the device job table and the
// block -> job map for the plan's tile width.
int build_tables(rbsm_plan *plan, const rbsm_job *jobs, int32_t n_jobs, bool keep_layout) {
    const char *fn = keep_layout ? "rbsm_plan_update" : "rbsm_plan_create";
    if (!jobs || n_jobs < 1 || n_jobs > 65535) return fail(RBSM_ERR_INVALID_ARG, "%s: need 1..65535 jobs", fn);
    if (keep_layout && (size_t)n_jobs != plan->jobs.size())
        return fail(RBSM_ERR_INVALID_ARG, "%s: job count differs from the plan", fn);
    std::vector<JobDev> dev(n_jobs);
    std::vector<uint16_t> block_job;
    int64_t base = 0, frags = 0;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const rbsm_job &J = jobs[j];
        if (J.mode != 0 && J.mode != 1) return fail(RBSM_ERR_INVALID_ARG, "%s: job mode must be 0 or 1", fn);
        MapView mv;
        const int st = validate(fn, J.shadow_map, J.frags, J.n, &J.params, J.out, J.mode == 0 ? 1 : 4, false, &mv);
        if (st != RBSM_OK) return st;
        if (keep_layout && (J.n != plan->jobs[j].n || J.params.view_width != plan->jobs[j].params.view_width))
            return fail(RBSM_ERR_INVALID_ARG, "%s: a job's n or view_width differs from the plan", fn);
        const JobLayout L = job_layout(J.n, J.params.view_width, plan->tune.tile_w);
        JobDev &D = dev[j];
        D.m = mv;
        D.frags = J.frags;
        D.out = J.out;
        D.n = J.n;
        D.vw = L.vw;
        D.tiles_x = L.tiles_x;
        D.tile_base = base;
        D.bias = J.params.depth_bias;
        D.maxd = J.params.max_dist;
        D.mode = J.mode;
        D.vec_ok = ((uintptr_t)J.frags % 16 == 0) && ((uintptr_t)J.out % (J.mode == 0 ? 4 : 16) == 0) &&
                   (L.vw % 4 == 0);
        for (int64_t b = 0; b < L.tiles; ++b) block_job.push_back((uint16_t)j);
        base += L.tiles;
        frags += J.n;
    }
    // outputs must not overlap each other or any input of any job
    for (int32_t a = 0; a < n_jobs; ++a) {
        const size_t ob = (size_t)jobs[a].n * (jobs[a].mode == 0 ? 1 : 4);
        for (int32_t b = 0; b < n_jobs; ++b) {
            if (jobs[a].n == 0 || jobs[b].n == 0) continue;
            const rbsm_params &P = jobs[b].params;
            const size_t mb = ((size_t)(P.height - 1) * (size_t)P.pitch + (size_t)P.width) * 4u;
            if (overlaps(jobs[a].out, ob, jobs[b].shadow_map, mb) ||
                overlaps(jobs[a].out, ob, jobs[b].frags, (size_t)jobs[b].n * 12u) ||
                (a != b && overlaps(jobs[a].out, ob, jobs[b].out, (size_t)jobs[b].n * (jobs[b].mode == 0 ? 1 : 4))))
                return fail(RBSM_ERR_INVALID_ARG, "%s: a job output overlaps another array", fn);
        }
    }
    if (base > ((int64_t)1 << 24)) return fail(RBSM_ERR_INVALID_ARG, "%s: more than 2^24 tiles", fn);
    if (!keep_layout || base != plan->blocks) {
        free_tables(plan);
        if (hipMalloc(&plan->d_jobs, sizeof(JobDev) * (size_t)n_jobs) != hipSuccess ||
            hipMalloc(&plan->d_block_job, sizeof(uint16_t) * (size_t)std::max<int64_t>(base, 1)) != hipSuccess) {
            free_tables(plan);
            return fail(RBSM_ERR_HIP, "%s: could not allocate the job tables", fn);
        }
    }
    if (hipMemcpy(plan->d_jobs, dev.data(), sizeof(JobDev) * (size_t)n_jobs, hipMemcpyHostToDevice) != hipSuccess ||
        (base > 0 && hipMemcpy(plan->d_block_job, block_job.data(), sizeof(uint16_t) * (size_t)base,
                               hipMemcpyHostToDevice) != hipSuccess))
        return fail(RBSM_ERR_HIP, "%s: could not upload the job tables", fn);
    plan->jobs.assign(jobs, jobs + n_jobs);
    plan->blocks = base;
    plan->fragments = frags;
    return RBSM_OK;
}

void launch_batch(const rbsm_plan *p, hipStream_t stream) {
    if (p->blocks == 0) return;
    const dim3 grid((unsigned)p->blocks), block(kT);
    const size_t lds = (size_t)p->tune.lds_cap * sizeof(float);
    switch (p->tune.tile_w) {
        case 16:
            hipLaunchKernelGGL(batch_kernel<16>, grid, block, lds, stream, p->d_jobs, p->d_block_job, p->tune.apron,
                               p->tune.lds_cap);
            break;
        case 64:
            hipLaunchKernelGGL(batch_kernel<64>, grid, block, lds, stream, p->d_jobs, p->d_block_job, p->tune.apron,
                               p->tune.lds_cap);
            break;
        default:
            hipLaunchKernelGGL(batch_kernel<32>, grid, block, lds, stream, p->d_jobs, p->d_block_job, p->tune.apron,
                               p->tune.lds_cap);
            break;
    }
}

}  // namespace

extern "C" {

int rbsm_visibility(const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                    uint8_t *out_mask, hipStream_t stream) {
    MapView mv;
    const int st = validate("rbsm_visibility", shadow_map, frags, n, p, out_mask, 1, false, &mv);
    if (st != RBSM_OK) return st;
    if (n == 0) return RBSM_OK;
    launch_pass<true>(mv, frags, n, p->view_width, p->depth_bias, p->max_dist, kDefaultTile, out_mask, 4, stream);
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
        launch_pass<false>(mv, frags, n, p->view_width, p->depth_bias, p->max_dist, kDefaultTile, out_vis, 16,
                           stream);
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

rbsm_tuning rbsm_default_tuning(void) {
    rbsm_tuning t;
    t.tile_w = kDefaultTile.tile_w;
    t.apron = kDefaultTile.apron;
    t.lds_cap = kDefaultTile.cap;
    return t;
}

int rbsm_pass_tuned(int32_t mode, const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                    const rbsm_tuning *tune, void *out, hipStream_t stream) {
    if (mode != 0 && mode != 1) return fail(RBSM_ERR_INVALID_ARG, "rbsm_pass_tuned: mode must be 0 or 1");
    if (!tuning_ok(tune)) return fail(RBSM_ERR_INVALID_ARG, "rbsm_pass_tuned: invalid tuning");
    MapView mv;
    const int st = validate("rbsm_pass_tuned", shadow_map, frags, n, p, out, mode == 0 ? 1 : 4, false, &mv);
    if (st != RBSM_OK) return st;
    if (n == 0) return RBSM_OK;
    const TileConfig cfg{tune->tile_w, tune->apron, tune->lds_cap};
    if (mode == 0)
        launch_pass<true>(mv, frags, n, p->view_width, p->depth_bias, p->max_dist, cfg, out, 4, stream);
    else
        launch_pass<false>(mv, frags, n, p->view_width, p->depth_bias, p->max_dist, cfg, out, 16, stream);
    return launched("rbsm_pass_tuned");
}

int rbsm_plan_create(const rbsm_job *jobs, int32_t n_jobs, const rbsm_tuning *tune, rbsm_plan **plan) {
    if (!plan) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_create: plan is null");
    *plan = nullptr;
    if (tune && !tuning_ok(tune)) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_create: invalid tuning");
    rbsm_plan *p = new (std::nothrow) rbsm_plan();
    if (!p) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_create: out of host memory");
    p->tune = tune ? *tune : rbsm_default_tuning();
    (void)hipGetDevice(&p->device);
    const int st = build_tables(p, jobs, n_jobs, false);
    if (st != RBSM_OK) {
        free_tables(p);
        delete p;
        return st;
    }
    *plan = p;
    return RBSM_OK;
}

int rbsm_plan_update(rbsm_plan *plan, const rbsm_job *jobs, int32_t n_jobs) {
    if (!plan) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_update: plan is null");
    return build_tables(plan, jobs, n_jobs, true);
}

int rbsm_plan_launch(rbsm_plan *plan, hipStream_t stream) {
    if (!plan) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_launch: plan is null");
    if (plan->exec) {
        if (hipGraphLaunch(plan->exec, stream) != hipSuccess)
            return fail(RBSM_ERR_HIP, "rbsm_plan_launch: graph launch failed");
        return RBSM_OK;
    }
    launch_batch(plan, stream);
    return launched("rbsm_plan_launch");
}

int rbsm_plan_set_tuning(rbsm_plan *plan, const rbsm_tuning *tune) {
    if (!plan || !tuning_ok(tune)) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_set_tuning: invalid argument");
    drop_graph(plan);
    if (tune->tile_w != plan->tune.tile_w) {
        const rbsm_tuning old = plan->tune;
        plan->tune = *tune;
        const std::vector<rbsm_job> jobs = plan->jobs;
        const int st = build_tables(plan, jobs.data(), (int32_t)jobs.size(), false);
        if (st != RBSM_OK) {
            plan->tune = old;
            return st;
        }
    }
    plan->tune = *tune;
    return RBSM_OK;
}

int rbsm_plan_get_tuning(const rbsm_plan *plan, rbsm_tuning *tune) {
    if (!plan || !tune) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_get_tuning: null argument");
    *tune = plan->tune;
    return RBSM_OK;
}

int rbsm_plan_autotune(rbsm_plan *plan, hipStream_t stream, int32_t reps, rbsm_tuning *chosen) {
    if (!plan || reps < 1) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_autotune: invalid argument");
    drop_graph(plan);
    const int tws[] = {16, 32, 64};
    const int caps[] = {2048, 3072, 4096};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RBSM_ERR_HIP, "rbsm_plan_autotune: could not create events");
    rbsm_tuning best = plan->tune;
    float best_ms = 1e30f;
    int status = RBSM_OK;
    for (int tw : tws) {
        for (int cap : caps) {
            rbsm_tuning cand{tw, 1, cap};
            if ((status = rbsm_plan_set_tuning(plan, &cand)) != RBSM_OK) break;
            launch_batch(plan, stream);  // warm-up
            (void)hipEventRecord(e0, stream);
            for (int r = 0; r < reps; ++r) launch_batch(plan, stream);
            (void)hipEventRecord(e1, stream);
            if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) {
                status = fail(RBSM_ERR_HIP, "rbsm_plan_autotune: a timed launch failed");
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) {
                best_ms = ms;
                best = cand;
            }
        }
        if (status != RBSM_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != RBSM_OK) return status;
    if ((status = rbsm_plan_set_tuning(plan, &best)) != RBSM_OK) return status;
    if (chosen) *chosen = best;
    return RBSM_OK;
}

int rbsm_plan_capture(rbsm_plan *plan, hipStream_t stream) {
    if (!plan || !stream) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_capture: need a plan and a non-default stream");
    drop_graph(plan);
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(RBSM_ERR_HIP, "rbsm_plan_capture: could not begin capture");
    launch_batch(plan, stream);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(stream, &g) != hipSuccess || !g)
        return fail(RBSM_ERR_HIP, "rbsm_plan_capture: capture failed");
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(RBSM_ERR_HIP, "rbsm_plan_capture: could not instantiate the graph");
    }
    plan->graph = g;
    plan->exec = x;
    return RBSM_OK;
}

int64_t rbsm_plan_fragments(const rbsm_plan *plan) { return plan ? plan->fragments : -1; }

void rbsm_plan_destroy(rbsm_plan *plan) {
    if (!plan) return;
    drop_graph(plan);
    free_tables(plan);
    delete plan;
}

const char *rbsm_last_error(void) { return g_err; }

int32_t rbsm_abi_version(void) { return 100; }

}  // extern "C"
