// Main hard / RSMSS (radius 0) pass for gfx950: 2-D screen tiles whose
// light-space footprint is staged in LDS, edge fragments compacted with wave
// ballots, traversals run one lane per (edge fragment, direction) in blocks
// of steps read from global memory.  Included once, by rbsm.hip.
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
constexpr int kState = 128;        // edge fragments whose full state is kept in LDS
constexpr int kWalkFirst = 2;     // steps every walk takes before the unfinished ones are compacted
constexpr int kWalkSteps = 4;     // steps per block of a continued walk, all reads issued together
constexpr int kCont = 512;         // continued walks queued per tile (more finish where they are)

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

// Bounded traversal (Listing 3) of one walk, a range of its steps at a time in
// blocks of NB steps, every read of a block issued together.  The walk moves
// along one coordinate p (clamped to [0, pmax]); the other coordinate is fixed
// for the texel on the walk and for its two side neighbours (the texels of the
// shared-discontinuity test), so a reader maps p to three texel values.
// walk_range returns +k (the walk ends at step k) or -k (it leaves the
// discontinuity at step k) for the first stopping step in [k0, k1], or 0.
struct GlobalWalkReader {  // a map under 4 GiB in global memory
    const char *t;           // map base (uniform)
    unsigned c, a, b;        // byte offsets of the fixed coordinate
    unsigned step4;          // bytes per unit of p
    __device__ __forceinline__ void operator()(int p, float &tc, float &ta, float &tb) const {
        const unsigned x = (unsigned)p * step4;
        tc = *(const float *)(t + (c + x));
        ta = *(const float *)(t + (a + x));
        tb = *(const float *)(t + (b + x));
    }
};

template <int NB, class Reader>
__device__ __forceinline__ int walk_range(const Reader &rd3, int k0, int k1, int p0, int d, int pmax, float zb, bool s,
                                          bool chk_a, bool chk_b) {
    for (int k = k0; k <= k1; k += NB) {
        float tc[NB], ta[NB], tb[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int ku = min(k + u, k1);
            rd3(min(max(p0 + __mul24(ku, d), 0), pmax), tc[u], ta[u], tb[u]);
        }
        // bit u: step k+u ends the walk (a texel whose test differs from s:
        // (zb > T) == s), or stops it (ends it, or shares no discontinuity
        // direction with the fragment); the first stopping step decides
        unsigned endb = 0, stopb = 0;
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const bool end = (zb > tc[u]) == s;
            const bool share = (chk_a & ((zb > ta[u]) == s)) | (chk_b & ((zb > tb[u]) == s));
            endb |= (unsigned)end << u;
            stopb |= (unsigned)(end | !share) << u;
        }
        const int left = k1 - k + 1;
        stopb &= left >= NB ? (1u << NB) - 1u : (1u << left) - 1u;
        if (stopb != 0u) {
            const int u = __builtin_ctz(stopb);
            return (endb >> u) & 1u ? k + u : -(k + u);
        }
    }
    return 0;
}

// Workgroup-shared state of one tile (the staged texels live in the dynamic
// LDS array that follows it).
struct TileShared {
    int box[kT / 64][4];
    int16_t slot[kTileF];
    uint8_t sm[kTileF];    // bit 4: centre test, bits 0-3: discontinuity mask
    int qi[kState], qj[kState];
    float qz[kState], qfx[kState], qfy[kState];
    int8_t rd[kTileF][4];  // left, right, top, bottom
    int16_t cont[kCont];   // walks (4 e + direction) continued after their first steps
    int count, ncont;
};

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
//  4. one lane per (edge fragment, direction) takes the walk's first
//     kWalkFirst steps from global memory (L2); walks still running are
//     queued again and continued in blocks of kWalkSteps steps;
//  5. one lane per edge fragment normalizes, evaluates the visibility
//     function and stores.
// Staging, tile shape and queues only decide where texels are read from and
// by which lane: every result equals the per-fragment listing.
// MODE: 1 hard pass, 0 RSMSS, 2 either, chosen per call by hard_rt (one code
// path for workgroups of both modes in one launch).
template <int MODE, int TW>
__device__ __forceinline__ void process_tile(MapView m, const float *__restrict__ frags, int64_t n, int64_t vw,
                                             int64_t tiles_x, float bias, int maxd, int apron, int cap,
                                             int vec_ok, void *__restrict__ out_v, int64_t tile_id,
                                             TileShared &sh, float *s_tex, bool hard_rt = false) {
    const bool HARD = MODE == 2 ? hard_rt : MODE == 1;
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
        if (t == 0) {
            q_count = 0;
            sh.ncont = 0;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kT / 64; ++w) {
            imin = min(imin, s_box[w][0]); imax = max(imax, s_box[w][1]);
            jmin = min(jmin, s_box[w][2]); jmax = max(jmax, s_box[w][3]);
        }
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

    // walks, one lane per (fragment, direction), straight from global memory
    // (L2) in blocks of steps whose reads are issued together; staging the
    // walks' bands in LDS first measured slower.  Most walks stop within a
    // few steps, so every walk first takes kWalkFirst steps; the unfinished
    // ones are compacted into a queue and continued by as few waves as
    // possible instead of holding every wave that has one of them.
    const bool map_32 = (int64_t)m.pitch * m.H * 4 <= (int64_t)0xFFFFFFFFu;  // byte offsets fit 32 bits
    struct Walk {
        GlobalWalkReader r;
        int p0, d, pmax;
        float zb;
        bool s, chk_a, chk_b;
    };
    // walk `task` = 4 e + direction (0 left, 1 right, 2 top, 3 bottom)
    auto make_walk = [&](int task, int &i0, int &j0) -> Walk {
        const int e = task >> 2, dir = task & 3;
        float zb, fx, fy;
        state_of(e, i0, j0, zb, fx, fy);
        const unsigned sm = q_sm[e];
        Walk w;
        w.zb = zb;
        w.s = HARD || (sm & 16u) != 0;  // the hard pass queues lit fragments only
        const bool horiz = dir < 2;
        w.d = dir == 0 || dir == 3 ? -1 : 1;
        w.p0 = horiz ? i0 : j0;
        w.pmax = (horiz ? m.W : m.H) - 1;
        w.chk_a = horiz ? (sm & BIT_T) != 0 : (sm & BIT_L) != 0;
        w.chk_b = horiz ? (sm & BIT_B) != 0 : (sm & BIT_R) != 0;
        // the fixed coordinate of the walk's texel and of its side neighbours
        // (rows j0, j0+1, j0-1 of a horizontal walk; columns i0, i0-1, i0+1 of
        // a vertical one), clamped to the map
        const int fc = horiz ? clampi(j0, m.H) : clampi(i0, m.W);
        const int fa = horiz ? clampi(j0 + 1, m.H) : clampi(i0 - 1, m.W);
        const int fb = horiz ? clampi(j0 - 1, m.H) : clampi(i0 + 1, m.W);
        const unsigned fmul = horiz ? 4u * (unsigned)m.pitch : 4u;
        w.r.t = (const char *)m.t;
        w.r.c = (unsigned)fc * fmul;
        w.r.a = (unsigned)fa * fmul;
        w.r.b = (unsigned)fb * fmul;
        w.r.step4 = horiz ? 4u : 4u * (unsigned)m.pitch;
        return w;
    };
    const int first = min(kWalkFirst, maxd);
    for (int task = t; task < 4 * ne; task += kT) {
        int i0, j0;
        const Walk w = make_walk(task, i0, j0);
        int rd;
        if (map_32) {
            rd = walk_range<kWalkFirst>(w.r, 1, first, w.p0, w.d, w.pmax, w.zb, w.s, w.chk_a, w.chk_b);
            if (rd == 0 && first < maxd) {
                const int slot = atomicAdd(&sh.ncont, 1);
                if (slot < kCont) sh.cont[slot] = (int16_t)task;  // continued below
                else rd = walk_range<kWalkSteps>(w.r, first + 1, maxd, w.p0, w.d, w.pmax, w.zb, w.s, w.chk_a,
                                                 w.chk_b);
                if (slot < kCont) continue;
            }
            if (rd == 0) rd = -(maxd + 1);
        } else {
            // a map of 4 GiB or more: one step at a time, 64-bit addresses
            const int dir = task & 3;
            const int dx = dir == 0 ? -1 : (dir == 1 ? 1 : 0);
            const int dy = dir == 2 ? 1 : (dir == 3 ? -1 : 0);
            const int pa_x = dx != 0 ? 0 : -1, pa_y = dx != 0 ? 1 : 0;
            const int pb_x = dx != 0 ? 0 : 1, pb_y = dx != 0 ? -1 : 0;
            rd = -(maxd + 1);
            for (int k = 1; k <= maxd; ++k) {
                const int i = i0 + k * dx, j = j0 + k * dy;
                if (lit(w.zb, texel(m, i, j)) != w.s) {
                    rd = k;
                    break;
                }
                const bool share = (w.chk_a && lit(w.zb, texel(m, i + pa_x, j + pa_y)) != w.s) ||
                                   (w.chk_b && lit(w.zb, texel(m, i + pb_x, j + pb_y)) != w.s);
                if (!share) {
                    rd = -k;
                    break;
                }
            }
        }
        q_rd[task >> 2][task & 3] = (int8_t)rd;
    }
    __syncthreads();
    const int nc = min(sh.ncont, kCont);
    if (nc > 0) {
        for (int c = t; c < nc; c += kT) {
            const int task = sh.cont[c];
            int i0, j0;
            const Walk w = make_walk(task, i0, j0);
            const int rd = walk_range<kWalkSteps>(w.r, first + 1, maxd, w.p0, w.d, w.pmax, w.zb, w.s, w.chk_a,
                                                  w.chk_b);
            q_rd[task >> 2][task & 3] = (int8_t)(rd != 0 ? rd : -(maxd + 1));
        }
        __syncthreads();
    }

    // normalize, evaluate and store, one lane per edge fragment
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

// 8 waves per SIMD: 64 VGPRs (no spills) and, with the default LDS capacity,
// 19 KB of LDS let 8 workgroups share a CU, so a 1080p frame's 2,040 tiles
// are all resident at once (one round, no second prologue).
template <bool HARD, int TW>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(8, 8))) void tile_kernel(
    MapView m, const float *__restrict__ frags, int64_t n, int64_t vw, int64_t tiles_x, float bias, int maxd,
    int apron, int cap, int vec_ok, void *__restrict__ out_v) {
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
// (XCD-ordered) workgroup index to its job.  Each tile runs the steps of the
// single-view pass, so every output is bitwise the same; the mode is a
// per-workgroup value, so one code path serves both and fits 64 VGPRs.
template <int TW>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(8, 8))) void batch_kernel(const JobDev *__restrict__ jobs,
                                                   const uint16_t *__restrict__ block_job, int apron, int cap) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    const int64_t g = xcd_block(blockIdx.x, gridDim.x);
    const JobDev J = jobs[block_job[g]];
    const int64_t tile = g - J.tile_base;
    process_tile<2, TW>(J.m, J.frags, J.n, J.vw, J.tiles_x, J.bias, J.maxd, apron, cap, J.vec_ok, J.out, tile, sh,
                        s_tex, J.mode == 0);
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
