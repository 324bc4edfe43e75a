// Main hard / RSMSS (radius 0) pass for gfx950: 2-D screen tiles whose
// light-space footprint is staged in LDS, edge fragments compacted with wave
// ballots, traversals run one lane per (edge fragment, direction) from LDS
// bands.  Included once, by rbsm.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbsm.h"
#include "rbsm_device.hpp"

namespace rbsm {

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

typedef __attribute__((address_space(3))) float lds_float;  // a float in LDS

constexpr int kStageChunk = 8;  // texels per thread whose loads are in flight together

// Copy texels [y0, y0+h) x [x0, x0+w) of the map into dst (row-major, stride
// w), the workgroup's kT threads striding over the rectangle.  Each thread
// issues kStageChunk loads before its first LDS store, so a chunk of
// kT * kStageChunk texels costs one memory round trip, not one per texel.
__device__ __forceinline__ void stage_rect(const MapView &m, float *dst, int x0, int y0, int w, int h, int t) {
    const int area = w * h;
    int r = t / w, c = t % w;
    const int dr = kT / w, dc = kT % w;
    for (int base = 0; base < area; base += kT * kStageChunk) {
        float v[kStageChunk];
#pragma unroll
        for (int u = 0; u < kStageChunk; ++u) {
            const int idx = base + u * kT + t;
            v[u] = idx < area ? m.t[(int64_t)(y0 + r) * m.pitch + (x0 + c)] : 0.0f;
            r += dr;
            c += dc;
            if (c >= w) {
                c -= w;
                ++r;
            }
        }
#pragma unroll
        for (int u = 0; u < kStageChunk; ++u) {
            const int idx = base + u * kT + t;
            if (idx < area) dst[idx] = v[u];
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

        // centre and neighbour texels; the staged path reads through an LDS
        // address-space pointer so its loads stay ds_reads (a merged generic
        // pointer would make every read a 64-bit-addressed flat load)
        float tc[kF][5];  // left, centre, right, top, bottom
        if (st.on) {
            const lds_float *lt = (const lds_float *)s_tex;
#pragma unroll
            for (int f = 0; f < kF; ++f) {
                const int ti = min(max(ad[f].i0, 0), m.W - 1), tj = min(max(ad[f].j0, 0), m.H - 1);
                const int il = max(ti - 1, 0), ir = min(ti + 1, m.W - 1);
                const int jl = max(tj - 1, 0), jh = min(tj + 1, m.H - 1);
                const int rc = (tj - st.by0) * st.bw - st.bx0;
                const bool ok = valid[f];
                tc[f][0] = ok ? lt[rc + il] : 0.0f;
                tc[f][1] = ok ? lt[rc + ti] : 0.0f;
                tc[f][2] = ok ? lt[rc + ir] : 0.0f;
                tc[f][3] = ok ? lt[(jh - st.by0) * st.bw - st.bx0 + ti] : 0.0f;
                tc[f][4] = ok ? lt[(jl - st.by0) * st.bw - st.bx0 + ti] : 0.0f;
            }
        } else {
#pragma unroll
            for (int f = 0; f < kF; ++f) {
                const int ti = min(max(ad[f].i0, 0), m.W - 1), tj = min(max(ad[f].j0, 0), m.H - 1);
                const int il = max(ti - 1, 0), ir = min(ti + 1, m.W - 1);
                const int jl = max(tj - 1, 0), jh = min(tj + 1, m.H - 1);
                const float *row = m.t + (int64_t)tj * m.pitch;
                const bool ok = valid[f];
                tc[f][0] = ok ? row[il] : 0.0f;
                tc[f][1] = ok ? row[ti] : 0.0f;
                tc[f][2] = ok ? row[ir] : 0.0f;
                tc[f][3] = ok ? m.t[(int64_t)jh * m.pitch + ti] : 0.0f;
                tc[f][4] = ok ? m.t[(int64_t)jl * m.pitch + ti] : 0.0f;
            }
        }
        bool s[kF], edge[kF];
        unsigned m0[kF];
#pragma unroll
        for (int f = 0; f < kF; ++f) {
            const float zb = ad[f].zb;
            s[f] = lit(zb, tc[f][1]);
            m0[f] = ((lit(zb, tc[f][0]) != s[f]) ? BIT_L : 0u) | ((lit(zb, tc[f][2]) != s[f]) ? BIT_R : 0u) |
                    ((lit(zb, tc[f][3]) != s[f]) ? BIT_T : 0u) | ((lit(zb, tc[f][4]) != s[f]) ? BIT_B : 0u);
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

        // 5. walks, one lane per (fragment, direction): from the LDS band in
        //    blocks of kLdsSteps steps with all reads of a block issued
        //    together, or step by step from global memory when the band did
        //    not fit
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
            if (in_lds) {
                // blocks of kLdsSteps steps, all reads of a block issued together
                const lds_float *bl = (const lds_float *)band;
                for (int k = 1; k <= maxd; k += kLdsSteps) {
                    float tc[kLdsSteps], ta[kLdsSteps], tb[kLdsSteps];
#pragma unroll
                    for (int u = 0; u < kLdsSteps; ++u) {
                        const int ku = min(k + u, maxd);
                        const int i = i0 + ku * dx, j = j0 + ku * dy;
                        tc[u] = bl[(clampi(j, m.H) - by0) * bstride + clampi(i, m.W) - bx0];
                        ta[u] = bl[(clampi(j + pa_y, m.H) - by0) * bstride + clampi(i + pa_x, m.W) - bx0];
                        tb[u] = bl[(clampi(j + pb_y, m.H) - by0) * bstride + clampi(i + pb_x, m.W) - bx0];
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
            } else {
                // the band did not fit: one step at a time from global memory
                // (rare; kept simple so it does not set the kernel's registers)
                for (int k = 1; k <= maxd; ++k) {
                    const int i = i0 + k * dx, j = j0 + k * dy;
                    if (lit(zb, texel(m, i, j)) != s) {
                        rd = k;
                        break;
                    }
                    const bool share = (chk_a && lit(zb, texel(m, i + pa_x, j + pa_y)) != s) ||
                                       (chk_b && lit(zb, texel(m, i + pb_x, j + pb_y)) != s);
                    if (!share) {
                        rd = -k;
                        break;
                    }
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

inline bool tuning_ok(const rbsm_tuning *t) {
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

}  // namespace rbsm
