// Main hard / RSMSS (radius 0) pass for gfx950: 2-D screen tiles whose
// light-space footprint is staged in LDS, edge fragments compacted with wave
// ballots, traversals run one lane per (edge fragment, direction) in blocks
// of steps read from global memory.  A launch either gives every tile its own
// workgroup or keeps only resident workgroups, each looping over tiles with
// the next tile's fragments loading while it works on the current one.
// Included once, by rbsm.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

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

// Chunked XCD order: the launch's tiles are dealt to the 8 XCDs in chunks of
// 2^chunk_log2 consecutive tiles, round-robin, so every XCD gets a share of
// every part of the launch (a tile's cost varies several-fold between jobs:
// staged or not, edges or not), while the tiles of a chunk still share one
// L2.  chunk_log2 < 0: one contiguous range per XCD (xcd_block).  A bijection
// for any grid size: the last, partial round of chunks is split contiguously.
__device__ __forceinline__ int64_t xcd_chunked(int b, int nb, int chunk_log2) {
    if (chunk_log2 < 0) return xcd_block(b, nb);
    const int round = 8 << chunk_log2;
    const int full = nb >> (3 + chunk_log2);  // nb / round
    if (b >= full * round) return (int64_t)full * round + xcd_block(b - full * round, nb - full * round);
    const int x = b & 7, l = b >> 3;
    const int q = l >> chunk_log2, r = l & ((1 << chunk_log2) - 1);
    return ((int64_t)(q * 8 + x) << chunk_log2) + r;
}

// ---------------------------------------------------------------------------
// Main pass: 2-D screen tiles with their light-space footprint staged in LDS.
// ---------------------------------------------------------------------------

constexpr int kT = 256;            // threads per workgroup
constexpr int kF = 4;              // consecutive pixels per thread
constexpr int kTileF = kT * kF;    // fragments per tile
constexpr int kState = 128;        // edge fragments whose full state is kept in LDS
constexpr int kWalkFirst = 2;     // default: steps every walk takes before the unfinished ones are compacted
constexpr int kWalkSteps = 4;     // default: steps per block of a continued walk, all reads issued together
constexpr int kCont = 512;         // continued walks queued per tile (more finish where they are)

// Staged light-space footprint of one screen tile: the window of texels
// [bx0, bx0+bw) x [by0, by0+bh) around the tile's (clamped) fragment texels,
// grown by the apron even past the map's edge (clamped texels there), stored
// row-major with stride bw.
struct Staged {
    const float *lds;
    int bx0, by0, bw, bh;  // window origin (may be -apron) and size
    bool on;
    bool inside;           // every fragment texel lies in the map (no clamps needed)
};

__device__ __forceinline__ int clampi(int x, int n) { return min(max(x, 0), n - 1); }

typedef __attribute__((address_space(3))) float lds_float;  // a float in LDS

constexpr int kStageChunk = 8;  // texels per thread whose loads are in flight together
constexpr int kStageRows4 = 2;  // 4-texel row groups per thread whose loads are in flight together

// Copy the map window [x0, x0+w) x [y0, y0+h) into dst (row-major, stride w).
// The window may leave the map by the apron; positions outside it hold the
// clamped texel, so a staged texel's 4 neighbours are always at fixed offsets
// (+-1, +-w) with clamp-to-edge already applied.  Each thread issues
// kStageChunk loads before its first LDS store, so a chunk costs one memory
// round trip.
//  - a window at most kT texels wide in a map under 4 GiB: every thread owns
//    one column (its clamped x fixed) and kT / w rows per round; a texel costs
//    a 32-bit address add (a row clamp where the window leaves the map), a
//    row compare and an LDS address add;
//  - otherwise the threads stride over the window with clamped coordinates.
__device__ __forceinline__ void stage_rect(const MapView &m, float *dst, int x0, int y0, int w, int h, int t) {
    const int ng = (w + 3) >> 2;  // groups of 4 texels per window row
    if (ng <= kT && x0 >= 0 && x0 + 4 * ng <= m.W && y0 >= 0 && y0 + h <= m.H &&
        (int64_t)m.pitch * m.H <= (int64_t)(0xFFFFFFFFu / 4u)) {
        // inside the map with whole groups: every thread owns one group of
        // 4 columns (one 16-byte load per row, dword aligned) and every
        // (kT / ng)-th row; rows past the window re-read the thread's first
        // row and are not stored, columns past it are not stored
        const int rpr = kT / ng;
        const int r0 = t / ng, g = t - r0 * ng;
        if (r0 >= rpr) return;
        const char *base8 = (const char *)m.t;
        const unsigned pitch4 = 4u * (unsigned)m.pitch;
        const unsigned col4 = 4u * (unsigned)(x0 + 4 * g);
        const int c0 = 4 * g;
        for (int r = r0; r < h; r += rpr * kStageRows4) {
            f32x4u v[kStageRows4];
#pragma unroll
            for (int u = 0; u < kStageRows4; ++u) {
                const int row = r + u * rpr;
                const unsigned y = (unsigned)(y0 + (row < h ? row : r));
                v[u] = gld4u((const float *)(base8 + (y * pitch4 + col4)));
            }
#pragma unroll
            for (int u = 0; u < kStageRows4; ++u) {
                const int row = r + u * rpr;
                if (row < h) {
                    float *d = dst + row * w + c0;
                    d[0] = v[u].x;
                    if (c0 + 1 < w) d[1] = v[u].y;
                    if (c0 + 2 < w) d[2] = v[u].z;
                    if (c0 + 3 < w) d[3] = v[u].w;
                }
            }
        }
        return;
    }
    if (w <= kT && (int64_t)m.pitch * m.H <= (int64_t)(0xFFFFFFFFu / 4u)) {
        const int rpi = kT / w;  // rows per round
        const int c = t % w, r0 = t / w;
        if (r0 >= rpi) return;   // the kT % w threads without a column
        const char *base8 = (const char *)m.t;
        const unsigned pitch4 = 4u * (unsigned)m.pitch;
        const unsigned x4 = 4u * (unsigned)min(max(x0 + c, 0), m.W - 1);
        const int lstep = rpi * w;
        int li = r0 * w + c;
        if (y0 >= 0 && y0 + h <= m.H) {  // rows inside the map: no row clamp
            const unsigned dstep = (unsigned)rpi * pitch4;
            unsigned off = (unsigned)(y0 + r0) * pitch4 + x4;
            for (int r = r0; r < h; r += rpi * kStageChunk) {
                float v[kStageChunk];
#pragma unroll
                for (int u = 0; u < kStageChunk; ++u) {
                    // rows past the window re-read the first row (in bounds) and are not stored
                    const bool ok = r + u * rpi < h;
                    v[u] = gld((const float *)(base8 + (ok ? off + (unsigned)u * dstep : off)));
                }
#pragma unroll
                for (int u = 0; u < kStageChunk; ++u)
                    if (r + u * rpi < h) dst[li + u * lstep] = v[u];
                off += (unsigned)kStageChunk * dstep;
                li += kStageChunk * lstep;
            }
        } else {
            for (int r = r0; r < h; r += rpi * kStageChunk) {
                float v[kStageChunk];
#pragma unroll
                for (int u = 0; u < kStageChunk; ++u) {
                    const int y = min(max(y0 + r + u * rpi, 0), m.H - 1);  // rows past the window: clamped, not stored
                    v[u] = gld((const float *)(base8 + ((unsigned)y * pitch4 + x4)));
                }
#pragma unroll
                for (int u = 0; u < kStageChunk; ++u)
                    if (r + u * rpi < h) dst[li + u * lstep] = v[u];
                li += kStageChunk * lstep;
            }
        }
        return;
    }
    const int area = w * h;
    for (int base = 0; base < area; base += kT * kStageChunk) {
        float v[kStageChunk];
#pragma unroll
        for (int u = 0; u < kStageChunk; ++u) {
            const int idx = min(base + u * kT + t, area - 1);
            const int r = idx / w, c = idx - r * w;
            const int x = min(max(x0 + c, 0), m.W - 1), y = min(max(y0 + r, 0), m.H - 1);
            v[u] = gld(m.t + ((int64_t)y * m.pitch + x));
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
        tc = gld((const float *)(t + (c + x)));
        ta = gld((const float *)(t + (a + x)));
        tb = gld((const float *)(t + (b + x)));
    }
};

struct LdsWalkReader {  // the staged window in LDS (row stride bw)
    const lds_float *t;   // window base
    int c, a, b;          // window index of the fixed coordinate, less the moving one's origin
    int step;             // window index per unit of p
    __device__ __forceinline__ void operator()(int p, float &tc, float &ta, float &tb) const {
        const int x = p * step;
        tc = t[c + x];
        ta = t[a + x];
        tb = t[b + x];
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
    float qz[kState], qfx[kState], qfy[kState];  // sub-texel position: written by the walk phase
    int8_t rd[kTileF][4];  // left, right, top, bottom
    int16_t cont[kCont];   // walks (4 e + direction) continued after their first steps
    int count, ncont;
};

// Minimum over the 64 lanes of a wave, returned to every lane: a DPP
// reduction (rows of 16 by shifts, then the row broadcasts), 6 VALU
// instructions where a shuffle tree takes about 30.  The box reduction feeds
// it values in [-2^20, 2^20] or INT32_MAX, and negates only the former.
__device__ __forceinline__ int wave_min(int x) {
    x = min(x, __builtin_amdgcn_update_dpp(INT32_MAX, x, 0x111, 0xf, 0xf, false));  // row_shr:1
    x = min(x, __builtin_amdgcn_update_dpp(INT32_MAX, x, 0x112, 0xf, 0xf, false));  // row_shr:2
    x = min(x, __builtin_amdgcn_update_dpp(INT32_MAX, x, 0x114, 0xf, 0xf, false));  // row_shr:4
    x = min(x, __builtin_amdgcn_update_dpp(INT32_MAX, x, 0x118, 0xf, 0xf, false));  // row_shr:8
    x = min(x, __builtin_amdgcn_update_dpp(INT32_MAX, x, 0x142, 0xa, 0xf, false));  // row_bcast:15
    x = min(x, __builtin_amdgcn_update_dpp(INT32_MAX, x, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(x, 63);
}

// The thread index through an opaque copy: in a persistent loop nothing
// derived from it is hoisted out of a tile and held in registers across tiles
// (recomputing it per tile costs a few instructions; holding it costs VGPRs
// the tile needs).
__device__ __forceinline__ int opaque_tid() {
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    return t;
}

// Every fragment index a tile's threads form (padding pixels included) is
// below n + TH * vw + TW.  Below kIndex32 the tile runs in the 32-bit form:
// indices are 32-bit and buffers are addressed by unsigned 32-bit byte
// offsets from their base (12 bytes per fragment stay below 2^32), which
// takes about a twentieth of the pass's VALU instructions and the scalar
// registers of the 64-bit index pairs (those otherwise spill to VGPR lanes).
constexpr int64_t kIndex32 = (int64_t)1 << 28;

__host__ __device__ inline bool index32(int64_t n, int64_t vw, int tw) {
    return n + (int64_t)(kTileF / tw) * vw + tw < kIndex32;
}

// Element k of buffer p: in the 32-bit form (IX = int) an unsigned byte
// offset from the base.
template <class IX, class T>
__device__ __forceinline__ T *at(T *p, IX k) {
    if constexpr (sizeof(IX) == 4) {
        using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
        return reinterpret_cast<T *>(reinterpret_cast<C *>(p) + (unsigned)k * (unsigned)sizeof(T));
    } else {
        return p + k;
    }
}

// Where a thread's 4 pixels of tile `tile_id` sit: a TW x (1024/TW) tile of a
// row-major image of width vw (flat mode: vw = n, TW = 1024), each thread 4
// consecutive pixels of one row.  Tile and image counts stay below 2^31.
// IX = int: the caller has checked index32.  IX = int64_t: when every index
// is below 2^31 (a uniform test) the per-thread arithmetic is still 32-bit.
template <int TW, class IX = int64_t>
struct TilePos {
    IX tyi, txi, px0, k0;
    int avail;  // how many of the thread's 4 pixels are in the image (0..4)
    __device__ __forceinline__ TilePos(int64_t vw, int64_t n, int64_t tiles_x, int64_t tile_id, int t) {
        constexpr int TH = kTileF / TW;
        constexpr int LPR = TW / kF;
        tyi = (IX)((uint32_t)tile_id / (uint32_t)tiles_x);
        txi = (IX)(tile_id - (int64_t)tyi * tiles_x);
        if (sizeof(IX) == 4 || n + (int64_t)TH * vw + TW < ((int64_t)1 << 31)) {
            const int px = (int)txi * TW + (t % LPR) * kF;
            const int k = ((int)tyi * TH + t / LPR) * (int)vw + px;
            px0 = px;
            k0 = k;
            avail = max(min(min((int)vw - px, (int)n - k), kF), 0);
        } else {
            px0 = (IX)((int64_t)txi * TW + (int64_t)(t % LPR) * kF);
            k0 = (IX)(((int64_t)tyi * TH + t / LPR) * vw + px0);
            const int64_t lim = min(vw - (int64_t)px0, n - (int64_t)k0);
            avail = (int)max(min(lim, (int64_t)kF), (int64_t)0);
        }
    }
};

// Fragment loads of one thread for one tile: one 48-byte load (three 16-byte
// ones) when the 4 pixels are in range and aligned, else guarded 4-byte loads
// (zeros where a pixel lies outside the image).
template <int TW, class IX>
__device__ __forceinline__ void load_tile_frags(const float *__restrict__ frags, const TilePos<TW, IX> &P, int vec_ok,
                                                float (&fr)[3 * kF]) {
    bool valid[kF];
#pragma unroll
    for (int f = 0; f < kF; ++f) valid[f] = f < P.avail;
    if (vec_ok && valid[kF - 1]) {
        const float4 *p4 = reinterpret_cast<const float4 *>(at(frags, 3 * P.k0));
        const float4 a = gld4(p4), b = gld4(p4 + 1), c = gld4(p4 + 2);
        fr[0] = a.x; fr[1] = a.y; fr[2] = a.z; fr[3] = a.w;
        fr[4] = b.x; fr[5] = b.y; fr[6] = b.z; fr[7] = b.w;
        fr[8] = c.x; fr[9] = c.y; fr[10] = c.z; fr[11] = c.w;
    } else {
#pragma unroll
        for (int f = 0; f < kF; ++f) {
            const IX k3 = 3 * (P.k0 + f);
            fr[3 * f + 0] = valid[f] ? gld(at(frags, k3 + 0)) : 0.0f;
            fr[3 * f + 1] = valid[f] ? gld(at(frags, k3 + 1)) : 0.0f;
            fr[3 * f + 2] = valid[f] ? gld(at(frags, k3 + 2)) : 0.0f;
        }
    }
}

struct NoPrefetch {
    __device__ __forceinline__ void operator()() const {}
};

// One tile whose fragments fr the thread has already loaded:
//  1. the workgroup reduces the bounding box of the fragments' texels, grows
//     it by `apron` texels and, when it holds at most `cap` texels, copies it
//     into LDS with row-contiguous loads (else reads stay global);
//  2. centre and neighbour tests; fragments without a discontinuity (and, in
//     hard mode, shadowed ones) are final and stored at once;
//  3. edge fragments are compacted with wave ballots into an LDS queue that
//     keeps their texel, depth, sub-texel position, test and mask;
//  4. one lane per (edge fragment, direction) takes the walk's first WF
//     steps from global memory (L2) (with LW: up to WF steps in the staged
//     window first); walks still running are queued again and continued in
//     blocks of WB steps from global memory;
//  5. one lane per edge fragment normalizes, evaluates the visibility
//     function and stores.
// `prefetch` runs once, right after the box reduction, every thread of the
// workgroup calling it: the persistent kernels issue the next tile's fragment
// loads there, so they arrive while this tile is staged, tested and walked.
// Staging, tile shape, queues and walk blocking only decide where texels are
// read from and by which lane: every result equals the per-fragment listing.
// MODE: 1 hard pass, 0 RSMSS, 2 either, chosen per call by hard_rt (one code
// path for workgroups of both modes in one launch).
template <int MODE, int TW, int WF = kWalkFirst, int WB = kWalkSteps, bool LW = false, class Prefetch = NoPrefetch,
          class IX>
__device__ __forceinline__ void process_tile_loaded(MapView m, const float *__restrict__ frags, int64_t vw64,
                                                    float bias, int maxd, int apron,
                                                    int cap, int vec_ok, void *__restrict__ out_v,
                                                    const TilePos<TW, IX> &P, const float (&fr)[3 * kF], TileShared &sh,
                                                    float *s_tex, bool hard_rt, const Prefetch &prefetch) {
    const bool HARD = MODE == 2 ? hard_rt : MODE == 1;
    constexpr int TH = kTileF / TW;
    constexpr int LPR = TW / kF;
    auto &s_box = sh.box;
    auto &q_slot = sh.slot;
    auto &q_sm = sh.sm;
    auto &q_i = sh.qi;
    auto &q_j = sh.qj;
    auto &q_z = sh.qz;
    auto &q_rd = sh.rd;
    int &q_count = sh.count;

    const int t = opaque_tid();
    const int lane = t & 63, wave = t >> 6;
    const IX tyi = P.tyi, txi = P.txi, k0 = P.k0, vw = (IX)vw64;
    const unsigned long long below = (1ull << lane) - 1ull;  // lanes below this one (from the opaque index)

    Staged st;
    {
        bool valid[kF];
#pragma unroll
        for (int f = 0; f < kF; ++f) valid[f] = f < P.avail;
        const bool full = vec_ok && valid[kF - 1];

        // cap == 0: direct reads, no box and no staging.  The queue counters
        // are cleared before the first fragment value is used, so the
        // barrier overlaps the fragment loads.
        const bool direct = cap == 0;
        auto clear_queue = [&] {
            if (t == 0) {
                // t - t: zero made from the thread index, so a loop over tiles
                // does not hold a zero pair in registers across tiles
                const int zero = t - opaque_tid();
                q_count = zero;
                sh.ncont = zero;
            }
        };
        if (direct) {
            clear_queue();
            __syncthreads();
        }
        Addr ad[kF];
#pragma unroll
        for (int f = 0; f < kF; ++f) ad[f] = address(fr[3 * f], fr[3 * f + 1], fr[3 * f + 2], m.W, m.H, bias);
        st.lds = s_tex;
        st.on = false;
        st.inside = false;
        if (direct) {
            prefetch();
        } else {
            // the box of the unclamped texel indices (|i|, |j| <= 2^20), clamped
            // to the map once reduced: clamping is monotone, so the clamped
            // box is the box of the clamped indices.  The initial imax = -1
            // clamps to 0 like any negative index, and imin > imax marks a
            // tile without fragments.
            int imin = INT32_MAX, imax = -1, jmin = INT32_MAX, jmax = -1;
#pragma unroll
            for (int f = 0; f < kF; ++f)
                if (valid[f]) {
                    imin = min(imin, ad[f].i0); imax = max(imax, ad[f].i0);
                    jmin = min(jmin, ad[f].j0); jmax = max(jmax, ad[f].j0);
                }
            imin = wave_min(imin);
            imax = -wave_min(-imax);
            jmin = wave_min(jmin);
            jmax = -wave_min(-jmax);
            if (lane == 0) {
                s_box[wave][0] = imin; s_box[wave][1] = imax;
                s_box[wave][2] = jmin; s_box[wave][3] = jmax;
            }
            clear_queue();
            __syncthreads();
            prefetch();
#pragma unroll
            for (int w = 0; w < kT / 64; ++w) {
                imin = min(imin, s_box[w][0]); imax = max(imax, s_box[w][1]);
                jmin = min(jmin, s_box[w][2]); jmax = max(jmax, s_box[w][3]);
            }
            // the box is the same in every lane: as wave-uniform values the
            // window and the staged / unstaged choice become scalar code and
            // uniform branches (the reads of one path then never wait for
            // reads the other path might have issued)
            imin = __builtin_amdgcn_readfirstlane(imin);
            imax = __builtin_amdgcn_readfirstlane(imax);
            jmin = __builtin_amdgcn_readfirstlane(jmin);
            jmax = __builtin_amdgcn_readfirstlane(jmax);
            const bool any = imin <= imax;
            // every fragment texel inside the map: the tests need no clamps
            st.inside = imin >= 0 && imax <= m.W - 1 && jmin >= 0 && jmax <= m.H - 1;
            imin = min(max(imin, 0), m.W - 1);
            imax = min(max(imax, 0), m.W - 1);
            jmin = min(max(jmin, 0), m.H - 1);
            jmax = min(max(jmax, 0), m.H - 1);
            st.bx0 = imin - apron;
            st.by0 = jmin - apron;
            st.bw = imax - imin + 1 + 2 * apron;
            st.bh = jmax - jmin + 1 + 2 * apron;
            st.on = any && (int64_t)st.bw * st.bh <= (int64_t)cap;
            if (st.on) stage_rect(m, s_tex, st.bx0, st.by0, st.bw, st.bh, t);
            __syncthreads();
        }

        // centre and neighbour texels; the staged path reads through an LDS
        // address-space pointer so its loads stay ds_reads (a merged generic
        // pointer would make every read a 64-bit-addressed flat load)
        float tc[kF][5];  // left, centre, right, top, bottom
        if (st.on) {
            // the window holds every fragment texel with a ring of at least
            // one texel, clamped at the map's edge: neighbours at +-1, +-bw
            const lds_float *lt = (const lds_float *)s_tex;
            auto read5 = [&](int f, int ti, int tj) {
                // 24-bit multiply: the row is below the window height and bw below 2^14
                const int c = valid[f] ? __mul24(tj - st.by0, st.bw) + (ti - st.bx0) : st.bw + 1;
                tc[f][0] = lt[c - 1];
                tc[f][1] = lt[c];
                tc[f][2] = lt[c + 1];
                tc[f][3] = lt[c + st.bw];
                tc[f][4] = lt[c - st.bw];
            };
            if (st.inside) {
#pragma unroll
                for (int f = 0; f < kF; ++f) read5(f, ad[f].i0, ad[f].j0);
            } else {
#pragma unroll
                for (int f = 0; f < kF; ++f)
                    read5(f, min(max(ad[f].i0, 0), m.W - 1), min(max(ad[f].j0, 0), m.H - 1));
            }
        } else {
            // the form of the reads is decided once per tile (uniform
            // branches around every fragment's reads), so the reads of all
            // kF fragments are in flight together
            int ti[kF], tj[kF];
#pragma unroll
            for (int f = 0; f < kF; ++f) {
                ti[f] = min(max(ad[f].i0, 0), m.W - 1);
                tj[f] = min(max(ad[f].j0, 0), m.H - 1);
            }
            const bool off32 = (int64_t)m.pitch * m.H <= (int64_t)(0xFFFFFFFFu / 4u);
            if (off32 && m.W >= 3) {  // 32-bit byte offsets from the map's base
                const char *base8 = (const char *)m.t;
                const unsigned pitch4 = 4u * (unsigned)m.pitch;
                f32x3 t3[kF];
                int sc[kF];
#pragma unroll
                for (int f = 0; f < kF; ++f) {
                    // left, centre and right in one 12-byte load: the clamped
                    // triple starts at column max(ti-1, 0), at most W-3 (at
                    // the map's left or right edge the centre or the right
                    // texel is the clamp)
                    const unsigned c3 = (unsigned)min(max(ti[f] - 1, 0), m.W - 3);
                    sc[f] = ti[f] - (int)c3;  // 0 (ti = 0), 1, or 2 (ti = W-1)
                    t3[f] = gld3((const float *)(base8 + (__umul24((unsigned)tj[f], pitch4) + 4u * c3)));
                    const int jl = max(tj[f] - 1, 0), jh = min(tj[f] + 1, m.H - 1);
                    // 24-bit multiplies: rows below 2^16, pitch4 below 2^18
                    tc[f][3] = gld((const float *)(base8 + (__umul24((unsigned)jh, pitch4) + 4u * (unsigned)ti[f])));
                    tc[f][4] = gld((const float *)(base8 + (__umul24((unsigned)jl, pitch4) + 4u * (unsigned)ti[f])));
                }
#pragma unroll
                for (int f = 0; f < kF; ++f) {
                    tc[f][0] = sc[f] == 2 ? t3[f].y : t3[f].x;
                    tc[f][1] = sc[f] == 0 ? t3[f].x : (sc[f] == 1 ? t3[f].y : t3[f].z);
                    tc[f][2] = sc[f] == 0 ? t3[f].y : t3[f].z;
                }
            } else {
#pragma unroll
                for (int f = 0; f < kF; ++f) {
                    const int il = max(ti[f] - 1, 0), ir = min(ti[f] + 1, m.W - 1);
                    const int jl = max(tj[f] - 1, 0), jh = min(tj[f] + 1, m.H - 1);
                    const float *row = m.t + (int64_t)tj[f] * m.pitch;
                    tc[f][0] = gld(row + il);
                    tc[f][1] = gld(row + ti[f]);
                    tc[f][2] = gld(row + ir);
                    tc[f][3] = gld(m.t + ((int64_t)jh * m.pitch + ti[f]));
                    tc[f][4] = gld(m.t + ((int64_t)jl * m.pitch + ti[f]));
                }
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
                gst(reinterpret_cast<uint32_t *>(at(out, k0)), packed);
            } else {
#pragma unroll
                for (int f = 0; f < kF; ++f)
                    if (valid[f] && !edge[f]) gst(at(out, k0 + f), (uint8_t)(s[f] ? 1 : 0));
            }
        } else {
            float *out = static_cast<float *>(out_v);
            if (full && !any_edge) {
                gst4(reinterpret_cast<float4 *>(at(out, k0)),
                    make_float4(s[0] ? 1.0f : 0.0f, s[1] ? 1.0f : 0.0f, s[2] ? 1.0f : 0.0f, s[3] ? 1.0f : 0.0f));
            } else {
#pragma unroll
                for (int f = 0; f < kF; ++f)
                    if (valid[f] && !edge[f]) gst(at(out, k0 + f), s[f] ? 1.0f : 0.0f);
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
            base = __builtin_amdgcn_readfirstlane(base);  // every lane is active here: lane 0's value
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
    auto frag_of = [&](int e) -> IX {
        const int slot = q_slot[e];
        const int owner = slot >> 2, f = slot & 3;
        return (tyi * TH + owner / LPR) * vw + txi * TW + (IX)(owner % LPR) * kF + f;
    };
    // texel and biased depth of queue entry e (from LDS, or recomputed past
    // kState); the sub-texel position, needed only by the last step, is
    // recomputed there from the fragment, so it is not held in registers
    // through the neighbour tests
    auto state_of = [&](int e, int &i0, int &j0, float &zb) {
        if (e < kState) {
            i0 = q_i[e]; j0 = q_j[e]; zb = q_z[e];
        } else {
            const IX k3 = 3 * frag_of(e);
            const Addr b = address(gld(at(frags, k3)), gld(at(frags, k3 + 1)), gld(at(frags, k3 + 2)), m.W, m.H, bias);
            i0 = b.i0; j0 = b.j0; zb = b.zb;
        }
    };

    // walks, one lane per (fragment, direction), from global memory (L2) in
    // blocks of steps whose reads are issued together (with LW, the first
    // steps that lie in the staged window read it instead; staging extra
    // bands for the walks measured slower).  Most walks stop within a few
    // steps, so every walk first takes WF steps (with LW, up to WF more past
    // the window); the unfinished ones are compacted into a queue and
    // continued by as few waves as possible instead of holding every wave
    // that has one of them.
    const bool map_32 = (int64_t)m.pitch * m.H * 4 <= (int64_t)0xFFFFFFFFu;  // byte offsets fit 32 bits
    struct Walk {
        GlobalWalkReader r;
        int p0, d, pmax;
        float zb;
        bool s, chk_a, chk_b;
    };
    struct WalkLds {
        LdsWalkReader l;
        int kin;  // steps 1..kin lie in the staged window
    };
    // walk `task` = 4 e + direction (0 left, 1 right, 2 top, 3 bottom); with
    // LW, lw (if given) receives its reader of the staged window
    auto make_walk = [&](int task, int &i0, int &j0, WalkLds *lw) -> Walk {
        const int e = task >> 2, dir = task & 3;
        float zb;
        state_of(e, i0, j0, zb);
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
        // The walk's clamped positions move monotonically away from the
        // fragment's clamped texel, which lies in the box: they stay in the
        // window [lo, hi] up to step kin >= 1 (every step when the window
        // reaches the map's edge on that side).  The fixed coordinates are
        // within one texel of the box, inside the apron.
        if constexpr (LW) {
            if (lw) {
                lw->kin = 0;
                if (st.on) {
                    const int lo = horiz ? st.bx0 : st.by0;
                    const int hi = lo + (horiz ? st.bw : st.bh) - 1;
                    const int kin = w.d > 0 ? (hi >= w.pmax ? maxd : hi - w.p0) : (lo <= 0 ? maxd : w.p0 - lo);
                    lw->kin = min(kin, maxd);
                    lw->l.t = (const lds_float *)s_tex;
                    if (horiz) {
                        lw->l.c = (fc - st.by0) * st.bw - st.bx0;
                        lw->l.a = (fa - st.by0) * st.bw - st.bx0;
                        lw->l.b = (fb - st.by0) * st.bw - st.bx0;
                        lw->l.step = 1;
                    } else {
                        lw->l.c = fc - st.bx0 - st.by0 * st.bw;
                        lw->l.a = fa - st.bx0 - st.by0 * st.bw;
                        lw->l.b = fb - st.bx0 - st.by0 * st.bw;
                        lw->l.step = st.bw;
                    }
                }
            }
        }
        return w;
    };
    const int first = min(WF, maxd);
    for (int task = t; task < 4 * ne; task += kT) {
        // the left walk's lane also reads the fragment's (u, v) for the last
        // step, in the same round trip as its walk's first reads
        const int e_uv = task >> 2;
        const bool uv = (task & 3) == 0 && e_uv < kState;
        float u = 0.0f, v = 0.0f;
        if (uv) {
            const IX k3 = 3 * frag_of(e_uv);
            u = gld(at(frags, k3));
            v = gld(at(frags, k3 + 1));
        }
        int i0, j0;
        WalkLds wl;
        const Walk w = make_walk(task, i0, j0, LW ? &wl : nullptr);
        int rd;
        bool queued = false;  // continued after the barrier
        if (map_32) {
            int kg = first;  // the last step taken before the continuation
            if constexpr (LW) {
                // up to WF steps in the window, then up to WF from global memory
                const int kl = min(wl.kin, first);
                rd = st.on ? walk_range<WF>(wl.l, 1, kl, w.p0, w.d, w.pmax, w.zb, w.s, w.chk_a, w.chk_b) : 0;
                kg = min(kl + WF, maxd);
                if (rd == 0) rd = walk_range<WF>(w.r, kl + 1, kg, w.p0, w.d, w.pmax, w.zb, w.s, w.chk_a, w.chk_b);
            } else {
                rd = walk_range<WF>(w.r, 1, first, w.p0, w.d, w.pmax, w.zb, w.s, w.chk_a, w.chk_b);
            }
            if (rd == 0 && kg < maxd) {
                const int slot = atomicAdd(&sh.ncont, 1);
                queued = slot < kCont;
                if (queued) sh.cont[slot] = (int16_t)task;
                else rd = walk_range<WB>(w.r, kg + 1, maxd, w.p0, w.d, w.pmax, w.zb, w.s, w.chk_a, w.chk_b);
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
        if (!queued) q_rd[task >> 2][task & 3] = (int8_t)rd;
        if (uv) {
            const Addr b = address(u, v, 0.0f, m.W, m.H, bias);
            sh.qfx[e_uv] = b.fx;
            sh.qfy[e_uv] = b.fy;
        }
    }
    __syncthreads();
    const int nc = min(sh.ncont, kCont);
    if (nc > 0) {
        for (int c = t; c < nc; c += kT) {
            const int task = sh.cont[c];
            int i0, j0;
            WalkLds wl;
            const Walk w = make_walk(task, i0, j0, LW ? &wl : nullptr);
            const int kg = LW ? min(min(wl.kin, first) + WF, maxd) : first;
            const int rd = walk_range<WB>(w.r, kg + 1, maxd, w.p0, w.d, w.pmax, w.zb, w.s, w.chk_a, w.chk_b);
            q_rd[task >> 2][task & 3] = (int8_t)(rd != 0 ? rd : -(maxd + 1));
        }
        __syncthreads();
    }

    // normalize, evaluate and store, one lane per edge fragment
    for (int e = t; e < ne; e += kT) {
        const IX k = frag_of(e);
        float fx, fy;
        if (e < kState) {
            fx = sh.qfx[e];
            fy = sh.qfy[e];
        } else {
            const Addr b = address(gld(at(frags, 3 * k)), gld(at(frags, 3 * k + 1)), 0.0f, m.W, m.H, bias);
            fx = b.fx;
            fy = b.fy;
        }
        const bool s = (q_sm[e] & 16u) != 0;
        const Axis axx = normalize_axis(q_rd[e][0], q_rd[e][1], fx);
        const Axis axy = normalize_axis(q_rd[e][3], q_rd[e][2], fy);
        if (HARD) gst(at(static_cast<uint8_t *>(out_v), k), (uint8_t)(vis_hard(axx, axy) != 0.0f ? 1 : 0));
        else gst(at(static_cast<float *>(out_v), k), vis_rsmss(s, axx, axy));
    }
}

// A tile whose fragments are loaded first (one workgroup per tile).  IX =
// int: the 32-bit form, which the launch has checked with index32.  LW: each
// walk first takes up to WF steps in the staged window, then up to WF from
// global memory, so a wave whose walks all stop in the window makes no global
// round trip (batched and serving launches, where many tiles share the GPU:
// a batched frame measured 2% faster; a single frame's launch, whose time is
// its slowest tiles, measured up to 8% slower in hard mode, so it keeps one
// block of global steps).
template <int MODE, int TW, int WF = kWalkFirst, int WB = kWalkSteps, class IX = int64_t, bool LW = false>
__device__ __forceinline__ void process_tile(MapView m, const float *__restrict__ frags, int64_t n, int64_t vw,
                                             int64_t tiles_x, float bias, int maxd, int apron, int cap,
                                             int vec_ok, void *__restrict__ out_v, int64_t tile_id,
                                             TileShared &sh, float *s_tex, bool hard_rt = false) {
    // the tile's pixel positions, computed once for the loads and the pass
    const TilePos<TW, IX> P(vw, n, tiles_x, tile_id, opaque_tid());
    float fr[3 * kF];
    load_tile_frags<TW>(frags, P, vec_ok, fr);
    process_tile_loaded<MODE, TW, WF, WB, LW>(m, frags, vw, bias, maxd, apron, cap, vec_ok, out_v, P, fr, sh, s_tex,
                                              hard_rt, NoPrefetch{});
}

// One job of a launch: a (view, light) pass over its own map, fragments and
// output, owning tiles [tile_base, tile_base + tiles) of the launch.
struct JobDev {
    MapView m;
    const float *frags;
    void *out;
    int64_t n, vw, tiles_x, tile_base;
    float bias;
    int maxd, vec_ok, mode;  // mode 0 hard, 1 RSMSS
};

// Persistent loop: the workgroup takes tiles g, g + G, g + 2G, ... of the
// launch (G = grid size, g its XCD-ordered index, so in every round each XCD
// works on one contiguous range of tiles and shares their texels in its L2).
// The next tile's job is read at the start of a tile and its fragments are
// loaded during the current one's staging, tests and walks.  job_of(tile)
// returns the tile's job (wave-uniform).
template <int MODE, int TW, int WF, int WB, class JobOf>
__device__ __forceinline__ void persistent_loop(const JobOf &job_of, int64_t tiles, int apron, int cap,
                                                TileShared &sh, float *s_tex) {
    const int64_t G = gridDim.x;
    int64_t g = xcd_block(blockIdx.x, gridDim.x);
    if (g >= tiles) return;
    JobDev J = job_of(g);
    float fr[3 * kF];
    load_tile_frags<TW>(J.frags, TilePos<TW>(J.vw, J.n, J.tiles_x, g - J.tile_base, opaque_tid()), J.vec_ok, fr);
    for (;;) {
        const int64_t gn = g + G;
        const bool more = gn < tiles;
        JobDev Jn = J;
        if (more) Jn = job_of(gn);
        float fn[3 * kF];
        auto pf = [&]() {
            if (more)
                load_tile_frags<TW>(Jn.frags, TilePos<TW>(Jn.vw, Jn.n, Jn.tiles_x, gn - Jn.tile_base, opaque_tid()),
                                    Jn.vec_ok, fn);
        };
        process_tile_loaded<MODE, TW, WF, WB>(J.m, J.frags, J.vw, J.bias, J.maxd, apron, cap, J.vec_ok, J.out,
                                              TilePos<TW>(J.vw, J.n, J.tiles_x, g - J.tile_base, opaque_tid()), fr,
                                              sh, s_tex, J.mode == 0, pf);
        if (!more) break;
        g = gn;
        J = Jn;
#pragma unroll
        for (int q = 0; q < 3 * kF; ++q) fr[q] = fn[q];
    }
}

// 8 waves per SIMD: 64 VGPRs (no spills) and, with the default LDS capacity,
// 19 KB of LDS let 8 workgroups share a CU, so a 1080p frame's 2,040 tiles
// are all resident at once (one round, no second prologue).
template <bool HARD, int TW, class IX>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(8, 8))) void tile_kernel(
    MapView m, const float *__restrict__ frags, int64_t n, int64_t vw, int64_t tiles_x, float bias, int maxd,
    int apron, int cap, int vec_ok, void *__restrict__ out_v, int chunk_log2) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    process_tile<HARD, TW, kWalkFirst, kWalkSteps, IX>(m, frags, n, vw, tiles_x, bias, maxd, apron, cap, vec_ok, out_v,
                                                       xcd_chunked(blockIdx.x, gridDim.x, chunk_log2), sh, s_tex);
}

// The same pass with resident workgroups looping over the tiles (the job is
// the kernel argument; tile_base 0).  The prefetched fragments and the loop
// need more registers than a one-shot tile: at 80 the loop spills, so the
// kernel runs at up to 96 VGPRs (5 waves per SIMD, 5 workgroups per CU).
template <bool HARD, int TW>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(5, 5))) void tile_persistent_kernel(
    const JobDev J, int64_t tiles, int apron, int cap) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    persistent_loop<HARD, TW, kWalkFirst, kWalkSteps>([&](int64_t) { return J; }, tiles, apron, cap, sh, s_tex);
}

// Batched pass: one workgroup per tile of any job; block_job maps the
// (XCD-ordered) workgroup index to its job.  Each tile runs the steps of the
// single-view pass, so every output is bitwise the same; the mode is a
// per-workgroup value, so one code path serves both and fits 64 VGPRs.  WF
// and WB are the walk blocking the autotuner searches.
template <int TW, int WF = kWalkFirst, int WB = kWalkSteps>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(8, 8))) void batch_kernel(const JobDev *__restrict__ jobs,
                                                   const uint16_t *__restrict__ block_job, int apron, int cap,
                                                   int chunk_log2) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    const int64_t g = xcd_chunked(blockIdx.x, gridDim.x, chunk_log2);
    const JobDev J = jobs[block_job[g]];
    const int64_t tile = g - J.tile_base;
    process_tile<2, TW, WF, WB, int64_t, true>(J.m, J.frags, J.n, J.vw, J.tiles_x, J.bias, J.maxd, apron, cap,
                                               J.vec_ok, J.out, tile, sh, s_tex, J.mode == 0);
}

// Batched pass with its job records in the kernel arguments: a workgroup
// finds its job from the jobs' first tiles (arg_job) and reads the record
// with scalar loads from the argument segment, which every workgroup
// reads and so stays in the scalar and L2 caches, instead of two dependent
// loads of device tables (the tile's job index, then the job record; about
// 1.3 us before a workgroup's fragment loads could start).  For batches of at
// most kArgJobsMax jobs with tiles, every one in the 32-bit form (index32).
struct JobArg {
    const float *t;        // map
    const float *frags;
    void *out;
    int32_t pitch, W, H;   // pitch in floats (< 2^31)
    int32_t n, vw, tiles_x, tile_base;
    float bias;
    int16_t maxd;
    uint8_t vec_ok, mode;  // mode 0 hard, 1 RSMSS
};

constexpr int kArgJobsMax = 48;

struct BatchArgs {
    int32_t first[kArgJobsMax];  // first tile of each job, increasing; INT32_MAX past the last job
    JobArg jobs[kArgJobsMax];
};

// The job of launch tile g: the last job whose first tile is at or below g
// (first tiles increase strictly; a launch has fewer than 2^24 tiles; g is
// wave-uniform).  Two rounds of scalar loads from the argument segment, where
// a binary search would chain five: every eighth first tile picks the group of
// eight, then the group's first tiles pick the job.
__device__ __forceinline__ int arg_job(const BatchArgs &a, int64_t g) {
    static_assert(kArgJobsMax % 8 == 0, "groups of eight jobs");
    const int g32 = __builtin_amdgcn_readfirstlane((int)g);
    int b = 0;
#pragma unroll
    for (int r = 8; r < kArgJobsMax; r += 8) b = a.first[r] <= g32 ? r : b;
    int j = b;
#pragma unroll
    for (int r = 1; r < 8; ++r) j = a.first[b + r] <= g32 ? b + r : j;
    return j;
}

template <int TW, int WF, int WB>
__device__ __forceinline__ void arg_tile(const BatchArgs &a, int64_t g, int apron, int cap, TileShared &sh,
                                         float *s_tex) {
    const JobArg &J = a.jobs[arg_job(a, g)];
    MapView m;
    m.t = J.t;
    m.pitch = J.pitch;
    m.W = J.W;
    m.H = J.H;
    process_tile<2, TW, WF, WB, int, true>(m, J.frags, J.n, J.vw, J.tiles_x, J.bias, J.maxd, apron, cap, J.vec_ok,
                                           J.out, g - J.tile_base, sh, s_tex, J.mode == 0);
}

template <int TW, int WF = kWalkFirst, int WB = kWalkSteps>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(8, 8))) void batch_arg_kernel(
    const BatchArgs a, int apron, int cap, int chunk_log2) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    arg_tile<TW, WF, WB>(a, xcd_chunked(blockIdx.x, gridDim.x, chunk_log2), apron, cap, sh, s_tex);
}

// The same pass with resident workgroups taking tiles from queues: one
// counter per XCD (workgroup b runs on XCD b mod 8) hands out that XCD's
// virtual blocks x, x + 8, x + 16, ... in order, and xcd_chunked maps them to
// tiles, so every XCD works through its own chunks (L2 locality) while its
// workgroups balance dynamically.  Thread 0 fetches the next index while the
// workgroup works on the current tile.  Each counter is fetched once per
// virtual block plus once per workgroup that stops; the fetch that returns
// the last of those values is the last use of the counter in the launch, and
// its workgroup clears it for the next launch (graph replays included).
template <int TW>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(8, 8))) void batch_arg_queue_kernel(
    const BatchArgs a, int tiles, int apron, int cap, int chunk_log2, int *__restrict__ counters) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    __shared__ int s_next;
    const int x = blockIdx.x & 7;
    const int n_x = (tiles - x + 7) >> 3;            // virtual blocks x + 8k below tiles
    const int g_x = ((int)gridDim.x - x + 7) >> 3;   // workgroups with b mod 8 == x
    const int last = n_x + g_x - 1;                  // the counter's final value handed out
    int *ctr = counters + 16 * x;                    // counters 64 bytes apart
    if (threadIdx.x == 0) s_next = atomicAdd(ctr, 1);
    __syncthreads();
    int k = s_next;
    while (k < n_x) {
        int pending = 0;
        if (threadIdx.x == 0) pending = atomicAdd(ctr, 1);  // the next index, in flight during this tile
        arg_tile<TW, kWalkFirst, kWalkSteps>(a, xcd_chunked(8 * k + x, tiles, chunk_log2), apron, cap, sh, s_tex);
        __syncthreads();  // the tile's shared state is free; every thread has read s_next
        if (threadIdx.x == 0) s_next = pending;
        __syncthreads();
        k = s_next;
    }
    if (threadIdx.x == 0 && k == last) atomicExch(ctr, 0);
}

// Batched pass with resident workgroups looping over the tiles of every job,
// the next tile's job and fragments read while the current tile is worked on;
// WF and WB are the walk blocking the autotuner searches.  Up to 96 VGPRs (5
// workgroups per CU), as tile_persistent_kernel.
template <int TW, int WF, int WB>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(5, 5))) void batch_persistent_kernel(
    const JobDev *__restrict__ jobs, const uint16_t *__restrict__ block_job, int64_t tiles, int apron, int cap) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    persistent_loop<2, TW, WF, WB>([&](int64_t g) { return jobs[block_job[g]]; }, tiles, apron, cap, sh, s_tex);
}

// Launch configuration of the main pass (defaults of the plain entry points).
struct TileConfig {
    int tile_w;      // 16, 32, 64 (2-D tiles) or 1024 (flat)
    int apron;       // texels staged beyond the fragments' texel box, >= 1
    int cap;         // LDS texel capacity per workgroup
    int persistent;  // 0: one workgroup per tile, 1: resident workgroups loop over tiles
    int chunk_log2;  // tiles dealt to XCDs in chunks of 2^chunk_log2; < 0: contiguous ranges
};

// Default: 32x32 tiles, a 1-texel apron, 2048 texels of LDS, one workgroup per
// tile, tiles dealt to XCDs in chunks of 8 (measured on frames streamed from
// HBM: a 4K RSMSS frame 12% faster than with one contiguous range of tiles per
// XCD, a 1080p hard frame the same).
constexpr TileConfig kDefaultTile{32, 1, 2048, 0, 3};
constexpr int kMaxChunkLog2 = 12;

// Persistent launches are built for the default walk blocking only.
inline bool tuning_ok(const rbsm_tuning *t) {
    if (!t) return false;
    const bool walk_default =
        (t->walk_first == 0 || t->walk_first == kWalkFirst) && (t->walk_block == 0 || t->walk_block == kWalkSteps);
    return (t->tile_w == 16 || t->tile_w == 32 || t->tile_w == 64) && t->apron >= 1 && t->apron <= 8 &&
           (t->lds_cap == 0 || (t->lds_cap >= 256 && t->lds_cap <= 12288)) &&
           (t->persistent == 0 || t->persistent == 1) &&
           (t->walk_first == 0 || t->walk_first == 1 || t->walk_first == 2 || t->walk_first == 4) &&
           (t->walk_block == 0 || t->walk_block == 4 || t->walk_block == 8) && t->xcd_chunk >= -1 &&
           t->xcd_chunk <= kMaxChunkLog2 && (t->persistent == 0 || walk_default);
}

// Resident workgroups of a persistent launch: the occupancy of `kernel` at
// `lds` bytes of dynamic LDS times the CUs of the current device.
inline int64_t resident_groups(const void *kernel, size_t lds) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kT, lds) != hipSuccess || per < 1) per = 1;
    return (int64_t)per * cus;
}

template <bool HARD, int TW>
void launch_tiles(const MapView &mv, const float *frags, int64_t n, int64_t vw, int64_t tiles_x, int64_t tiles,
                  float bias, int maxd, TileConfig cfg, int vec, void *out, hipStream_t stream) {
    const size_t lds = (size_t)cfg.cap * sizeof(float);
    if (cfg.persistent) {
        JobDev J{};
        J.m = mv;
        J.frags = frags;
        J.out = out;
        J.n = n;
        J.vw = vw;
        J.tiles_x = tiles_x;
        J.tile_base = 0;
        J.bias = bias;
        J.maxd = maxd;
        J.vec_ok = vec;
        J.mode = HARD ? 0 : 1;
        const void *k = reinterpret_cast<const void *>(&tile_persistent_kernel<HARD, TW>);
        const int64_t grid = std::min<int64_t>(tiles, resident_groups(k, lds));
        hipLaunchKernelGGL((tile_persistent_kernel<HARD, TW>), dim3((unsigned)grid), dim3(kT), lds, stream, J, tiles,
                           cfg.apron, cfg.cap);
    } else {
        if (index32(n, vw, TW))
            hipLaunchKernelGGL((tile_kernel<HARD, TW, int>), dim3((unsigned)tiles), dim3(kT), lds, stream, mv, frags,
                               n, vw, tiles_x, bias, maxd, cfg.apron, cfg.cap, vec, out, cfg.chunk_log2);
        else
            hipLaunchKernelGGL((tile_kernel<HARD, TW, int64_t>), dim3((unsigned)tiles), dim3(kT), lds, stream, mv,
                               frags, n, vw, tiles_x, bias, maxd, cfg.apron, cfg.cap, vec, out, cfg.chunk_log2);
    }
}

// Flat launches of few fragments (no screen layout): one lane per fragment,
// its five texels and its walks read from global memory (L2), the listing's
// steps per fragment (eval_texel), so every result equals the tile pass's.
// 1024-fragment tiles would leave most CUs idle (65,536 fragments make 64
// workgroups), and the texel box of scattered fragments spans the whole map,
// so staging would not happen anyway.
constexpr int64_t kFlatFragMax = (int64_t)1 << 20;

// One fragment's visibility (Listing 1) with the reads of each round issued
// together: its five texels, then the first two steps of all four walks
// (24 reads); walks still running continue in blocks of 4 steps.  The same
// texels and tests as eval_texel, whose walks take one dependent read per
// step, one walk after the other.  Maps under 4 GiB (32-bit byte offsets).
template <bool HARD>
__device__ __forceinline__ float eval_texel_blocked(const MapView &m, const Addr &a, int maxd) {
    const int i0 = a.i0, j0 = a.j0;
    const float zb = a.zb;
    const float t_c = texel(m, i0, j0), t_l = texel(m, i0 - 1, j0), t_r = texel(m, i0 + 1, j0);
    const float t_t = texel(m, i0, j0 + 1), t_b = texel(m, i0, j0 - 1);
    const bool s = lit(zb, t_c);
    if (HARD && !s) return 0.0f;
    const unsigned m0 = (lit(zb, t_l) != s ? BIT_L : 0u) | (lit(zb, t_r) != s ? BIT_R : 0u) |
                        (lit(zb, t_t) != s ? BIT_T : 0u) | (lit(zb, t_b) != s ? BIT_B : 0u);
    if (m0 == 0u) return s ? 1.0f : 0.0f;
    // walks 0 left, 1 right, 2 top, 3 bottom: the moving coordinate p, and the
    // fixed one of the walk's texel and its side neighbours (clamped)
    GlobalWalkReader rw[4];
    int p0[4], d[4], pmax[4];
    bool ca[4], cb[4];
#pragma unroll
    for (int dir = 0; dir < 4; ++dir) {
        const bool horiz = dir < 2;
        d[dir] = dir == 0 || dir == 3 ? -1 : 1;
        p0[dir] = horiz ? i0 : j0;
        pmax[dir] = (horiz ? m.W : m.H) - 1;
        ca[dir] = horiz ? (m0 & BIT_T) != 0 : (m0 & BIT_L) != 0;
        cb[dir] = horiz ? (m0 & BIT_B) != 0 : (m0 & BIT_R) != 0;
        const unsigned fmul = horiz ? 4u * (unsigned)m.pitch : 4u;
        rw[dir].t = (const char *)m.t;
        rw[dir].c = (unsigned)(horiz ? clampi(j0, m.H) : clampi(i0, m.W)) * fmul;
        rw[dir].a = (unsigned)(horiz ? clampi(j0 + 1, m.H) : clampi(i0 - 1, m.W)) * fmul;
        rw[dir].b = (unsigned)(horiz ? clampi(j0 - 1, m.H) : clampi(i0 + 1, m.W)) * fmul;
        rw[dir].step4 = horiz ? 4u : 4u * (unsigned)m.pitch;
    }
    const int first = min(2, maxd);
    float tc[4][2], ta[4][2], tb[4][2];
#pragma unroll
    for (int dir = 0; dir < 4; ++dir)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int ku = min(1 + u, first);
            rw[dir](min(max(p0[dir] + ku * d[dir], 0), pmax[dir]), tc[dir][u], ta[dir][u], tb[dir][u]);
        }
    int rd[4];
#pragma unroll
    for (int dir = 0; dir < 4; ++dir) {
        // bit u: step 1 + u ends the walk, or stops it (as in walk_range)
        unsigned endb = 0u, stopb = 0u;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const bool end = (zb > tc[dir][u]) == s;
            const bool share = (ca[dir] & ((zb > ta[dir][u]) == s)) | (cb[dir] & ((zb > tb[dir][u]) == s));
            endb |= (unsigned)end << u;
            stopb |= (unsigned)(end | !share) << u;
        }
        stopb &= first >= 2 ? 3u : 1u;
        const int u = __builtin_ctz(stopb | 4u);
        rd[dir] = stopb != 0u ? ((endb >> u) & 1u ? 1 + u : -(1 + u)) : 0;
    }
#pragma unroll
    for (int dir = 0; dir < 4; ++dir) {
        if (rd[dir] == 0 && first < maxd)
            rd[dir] = walk_range<4>(rw[dir], first + 1, maxd, p0[dir], d[dir], pmax[dir], zb, s, ca[dir], cb[dir]);
        if (rd[dir] == 0) rd[dir] = -(maxd + 1);
    }
    const Axis ax = normalize_axis(rd[0], rd[1], a.fx);
    const Axis ay = normalize_axis(rd[3], rd[2], a.fy);
    return HARD ? vis_hard(ax, ay) : vis_rsmss(s, ax, ay);
}

template <bool HARD>
__global__ __launch_bounds__(256) void frag_kernel(MapView m, const float *__restrict__ frags, int64_t n, float bias,
                                                   int maxd, void *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const Addr a = address(gld(frags + 3 * k), gld(frags + 3 * k + 1), gld(frags + 3 * k + 2), m.W, m.H, bias);
    const bool map_32 = (int64_t)m.pitch * m.H * 4 <= (int64_t)0xFFFFFFFFu;  // byte offsets fit 32 bits
    const float v = map_32 ? eval_texel_blocked<HARD>(m, a, maxd)
                           : eval_texel<HARD>(m, a.i0, a.j0, a.fx, a.fy, a.zb, maxd);
    if (HARD) gst(static_cast<uint8_t *>(out) + k, (uint8_t)(v != 0.0f ? 1 : 0));
    else gst(static_cast<float *>(out) + k, v);
}

template <bool HARD>
void launch_pass(const MapView &mv, const float *frags, int64_t n, int64_t view_width, float bias, int maxd,
                 TileConfig cfg, void *out, size_t out_align, hipStream_t stream) {
    if (view_width <= 0 && n <= kFlatFragMax) {
        hipLaunchKernelGGL((frag_kernel<HARD>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, mv, frags, n,
                           bias, maxd, out);
        return;
    }
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
    switch (tw) {
        case 16: launch_tiles<HARD, 16>(mv, frags, n, vw, tiles_x, tiles, bias, maxd, cfg, vec, out, stream); break;
        case 64: launch_tiles<HARD, 64>(mv, frags, n, vw, tiles_x, tiles, bias, maxd, cfg, vec, out, stream); break;
        case 1024: launch_tiles<HARD, 1024>(mv, frags, n, vw, tiles_x, tiles, bias, maxd, cfg, vec, out, stream); break;
        default: launch_tiles<HARD, 32>(mv, frags, n, vw, tiles_x, tiles, bias, maxd, cfg, vec, out, stream); break;
    }
}

}  // namespace rbsm
