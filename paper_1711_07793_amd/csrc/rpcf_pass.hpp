// RPCF: the RSMSS value averaged over the (2r+1)^2 texels around a
// fragment's texel, each evaluated with the fragment's own sub-texel position
// and depth (PCF over the filtered edge, Sec. 5.3).  Included once, by
// rbsm.hip.
//
// Every term of one fragment tests texels against the same depth, so the pass
// first turns the fragment's (2r+3)^2 neighbourhood into shadow-test bits, one
// 64-bit word per column (bit q <-> row j0-r-1+q).  A term's discontinuity
// mask (Eq. 2-3) is then a few shifts and XORs, and the terms without a
// discontinuity contribute their test result, so a column's worth of them is
// one popcount.  Only the terms with a discontinuity need traversals
// (Listing 3), normalization (Eq. 5) and Listing 5; their number varies
// wildly between fragments, so such terms of each pair of columns are compacted
// over the workgroup into an LDS list and evaluated one lane per term, keeping
// every lane busy instead of holding a wave for its busiest fragment.  A
// vertical traversal is first resolved on the fragment's column words, which
// hold the shadow-test bits of every row it can reach inside the kernel's
// window; horizontal ones take their first step from the neighbouring column's
// word and their second from a staged band.  The
// bands reach only a few steps past the window, which keeps the workgroup's
// LDS small enough for more of them per CU; the few longer traversals go on
// in global memory.
//
// The average is the exact mean of the (2r+1)^2 binary32 terms, rounded to
// binary32.  The terms are summed in binary64 (bit-word counts first, then the
// listed terms in list order) and divided by (2r+1)^2 once: for at most 4225
// terms in [0, 1] any binary64 summation order stays within 5e-13 of the exact
// mean, so the result is that mean rounded, up to one binary32 step at a
// near-tie.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbsm_device.hpp"
#include "tile_pass.hpp"

namespace rbsm {

constexpr int kRpcfT = 128;    // threads per workgroup, one fragment each
constexpr int kRpcfLaneBits = kRpcfT > 128 ? 8 : 7;  // lane field of a listed term
constexpr int kRpcfMaxR = 30;  // largest r whose 2r+3 rows fit one 64-bit column word
constexpr int kRpcfEnt = 512;  // terms with a discontinuity evaluated per round
constexpr int kRpcfReach = 3;  // traversal steps staged beyond the kernel radius

// Any radius: one lane per fragment, every term evaluated from global memory
// in the same a-major order, binary64 sum.
__global__ __launch_bounds__(256) void rpcf_naive_kernel(MapView m, const float *__restrict__ frags, int64_t n,
                                                         float bias, int maxd, int r, float *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const float u = frags[3 * k + 0], v = frags[3 * k + 1], z = frags[3 * k + 2];
    const Addr a = address(u, v, z, m.W, m.H, bias);
    double sum = 0.0;
    for (int da = -r; da <= r; ++da)
        for (int db = -r; db <= r; ++db)
            sum += (double)eval_texel<false>(m, a.i0 + da, a.j0 + db, a.fx, a.fy, a.zb, maxd);
    out[k] = (float)(sum / (double)((2 * r + 1) * (2 * r + 1)));
}

// Shadow-test bit of texel depth t for depth zb (Eq. 1): the sign bit of
// t - zb.  The difference is negative exactly when zb > t, except for
// t = -0, zb = +0 (difference -0, test lit) and for NaN; callers pass
// canon(t), which turns -0 into +0 and NaN (lit at every depth) into +inf.
__device__ __forceinline__ uint32_t push_bit(uint32_t w, float t, float zb) {
    return __builtin_amdgcn_alignbit(w, __float_as_uint(t - zb), 31);  // (w << 1) | sign
}

// Shadow-test bits of nb <= 64 texels: bit p is 1 when texel p, read by
// rd(p), is in shadow for depth zb.  Reads run in chunks of 8 up to the next
// multiple of 8, so rd must accept p that far; the bits at and above nb are
// cleared.
template <class Rd>
__device__ __forceinline__ uint64_t shadow_bits(Rd rd, int nb, float zb) {
    const int nb8 = (nb + 7) & ~7;
    uint32_t hi = 0, lo = 0;
    for (int c = nb8 - 8; c >= 32; c -= 8) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = rd(c + e);
#pragma unroll
        for (int e = 7; e >= 0; --e) hi = push_bit(hi, v[e], zb);
    }
    for (int c = min(nb8, 32) - 8; c >= 0; c -= 8) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = rd(c + e);
#pragma unroll
        for (int e = 7; e >= 0; --e) lo = push_bit(lo, v[e], zb);
    }
    const uint64_t all = ((uint64_t)hi << 32) | lo;
    return nb >= 64 ? all : all & ((1ull << nb) - 1ull);
}

__device__ __forceinline__ float canon(float t) { return t != t ? __builtin_inff() : t + 0.0f; }

typedef __attribute__((address_space(3))) const char lds_byte;

// Three texel lines of a staged band, read at one offset: the line a
// traversal moves along and its two side lines.
struct BandWalkReader {
    lds_byte *c, *a, *b;
    unsigned step;  // bytes per unit of p
    __device__ __forceinline__ void operator()(int p, float &tc, float &ta, float &tb) const {
        const unsigned x = step * (unsigned)p;
        tc = *(const lds_float *)(c + x);
        ta = *(const lds_float *)(a + x);
        tb = *(const lds_float *)(b + x);
    }
};

// A map line and its two side lines (rows c, a, b when horizontal, columns
// when not), read from global memory with clamp-to-edge.
struct MapLineReader {
    MapView m;
    int c, a, b;
    bool horiz;
    __device__ __forceinline__ void operator()(int p, float &tc, float &ta, float &tb) const {
        tc = horiz ? texel(m, p, c) : texel(m, c, p);
        ta = horiz ? texel(m, p, a) : texel(m, a, p);
        tb = horiz ? texel(m, p, b) : texel(m, b, p);
    }
};

// The first two steps of a horizontal traversal (Listing 3), with no branches
// so that the reads of all four traversals of a term can be in flight
// together: step 1 from w1, the shadow-test word of the neighbouring column in
// the walk's direction (bit q the term's row, q + 1 and q - 1 its side rows,
// bit 1 = in shadow), step 2 from the staged band.  +k / -k for the first
// stopping step, 0 if neither stops.
__device__ __forceinline__ int first_steps(const BandWalkReader &br, uint64_t w1, int q, int p0, int d, int maxd,
                                           float zb, bool s, bool chk_a, bool chk_b) {
    float c2, a2, b2;
    br(p0 + (maxd >= 2 ? 2 * d : d), c2, a2, b2);
    const uint64_t v = s ? w1 : ~w1;  // bit set: that texel's test differs from the term's
    const bool end1 = (v >> q) & 1ull, end2 = (zb > c2) == s;
    const bool share1 = (chk_a & (bool)((v >> (q + 1)) & 1ull)) | (chk_b & (bool)((v >> (q - 1)) & 1ull));
    const bool share2 = (chk_a & ((zb > a2) == s)) | (chk_b & ((zb > b2) == s));
    const int at2 = maxd >= 2 ? (end2 ? 2 : (share2 ? 0 : -2)) : 0;
    return end1 ? 1 : (share1 ? at2 : -1);
}

// Stop rows of a vertical traversal over the column words w (the term's
// column) and wl, wr (its left and right neighbours), bit 1 = in shadow: bit
// p of `end` is set where the texel of row p has a test that differs from the
// term's s (its bit equals s), and bit p of the result where the walk stops
// there: it ends, or no checked neighbour's texel differs from s.
__device__ __forceinline__ uint64_t stop_bits(uint64_t wl, uint64_t w, uint64_t wr, bool s, bool chk_l, bool chk_r,
                                              uint64_t &end) {
    const uint64_t flip = s ? 0ull : ~0ull;
    end = w ^ flip;
    const uint64_t share = (chk_l ? wl ^ flip : 0ull) | (chk_r ? wr ^ flip : 0ull);
    return end | ~share;
}

// A vertical traversal (Listing 3) of the term in row q of column word w, as
// far as the word reaches, up (rows q+1, ...) or down (rows q-1, ...): +k / -k
// for the first stopping step, -(maxd+1) when the walk runs out of steps
// inside the word, or 0 with `next` set to the first step past the word.
__device__ __forceinline__ int column_walk_up(uint64_t wl, uint64_t w, uint64_t wr, int q, int nbc, int maxd, bool s,
                                              bool chk_l, bool chk_r, int &next) {
    uint64_t end;
    const uint64_t stop = stop_bits(wl, w, wr, s, chk_l, chk_r, end);
    const int kn = min(nbc - 1 - q, maxd);  // steps inside the word, >= 1
    const uint64_t b = (stop >> (q + 1)) & ((1ull << kn) - 1ull);
    next = kn + 1;
    if (b != 0ull) {
        const int k = __builtin_ctzll(b) + 1;
        return (end >> (q + k)) & 1ull ? k : -k;
    }
    return kn == maxd ? -(maxd + 1) : 0;
}

__device__ __forceinline__ int column_walk_down(uint64_t wl, uint64_t w, uint64_t wr, int q, int maxd, bool s,
                                                bool chk_l, bool chk_r, int &next) {
    uint64_t end;
    const uint64_t stop = stop_bits(wl, w, wr, s, chk_l, chk_r, end);
    const int kn = min(q, maxd);  // steps inside the word (rows q-1 .. q-kn), >= 1
    const uint64_t b = stop & (((1ull << kn) - 1ull) << (q - kn));
    next = kn + 1;
    if (b != 0ull) {
        const int p = 63 - __builtin_clzll(b);  // nearest stopping row below q
        const int k = q - p;
        return (end >> p) & 1ull ? k : -k;
    }
    return kn == maxd ? -(maxd + 1) : 0;
}

// One workgroup per TW x (kRpcfT / TW) pixel tile of a row-major image of
// width vw (flat: vw = n, TW = kRpcfT).  With R = r + min(maxd, kRpcfReach),
// the texels every word and the first R - r steps of every traversal read lie
// in bands staged in LDS (with canon() applied) when they fit in `cap`
// texels; longer traversals go on in global memory:
//   H: rows of the fragments' texel box grown by r+1, columns grown by R
//      (row-major; horizontal traversals);
//   V (VB): columns grown by r+1, rows grown by R, stored transposed, each
//      column contiguous (column words and vertical traversals).
// Without V, column words read H down its columns (7 more rows staged for the
// chunked reads) and vertical traversals use H's rows: half the LDS, so more
// workgroups per CU, for slower column reads and a shorter vertical reach.
// Band coordinates are unclamped positions holding clamped texels, so no read
// clamps.  Otherwise everything reads global memory.  Requires 1 <= r <=
// kRpcfMaxR.  At most 128 VGPRs (4 waves per SIMD): the H-only form would
// take 154 (3 waves) and runs 5-12% faster held to 128, a few values spilled.
template <int TW, bool VB>
__global__ __launch_bounds__(kRpcfT) __attribute__((amdgpu_waves_per_eu(4))) void rpcf_kernel(MapView m, const float *__restrict__ frags, int64_t n,
                                                      int64_t vw, int64_t tiles_x, float bias, int maxd, int r,
                                                      int cap, float *__restrict__ out) {
    extern __shared__ float s_band[];
    __shared__ int s_red[kRpcfT / 64][4];
    __shared__ int s_wtot[2][kRpcfT / 64];
    __shared__ int s_fi[kRpcfT], s_fj[kRpcfT];
    __shared__ float s_ffx[kRpcfT], s_ffy[kRpcfT], s_fzb[kRpcfT];
    __shared__ uint32_t s_ent[kRpcfEnt];  // lane | q << LB | lit << (LB+6) | mask << (LB+7) | column << (LB+11)
    __shared__ float s_val[kRpcfEnt];
    __shared__ uint64_t s_cw[4][kRpcfT];  // this round's column words a-1 .. a+2 of each fragment
    constexpr int TH = kRpcfT / TW, LB = kRpcfLaneBits;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
    const int64_t px = txi * TW + (t % TW), py = tyi * TH + (t / TW);
    const int64_t k = py * vw + px;
    const bool valid = px < vw && k < n;
    Addr A{};
    if (valid) A = address(frags[3 * k + 0], frags[3 * k + 1], frags[3 * k + 2], m.W, m.H, bias);
    const int R = r + min(maxd, kRpcfReach);

    // texel box of the tile's fragments
    int b0 = valid ? A.i0 : INT32_MAX, b1 = valid ? -A.i0 : INT32_MAX;
    int b2 = valid ? A.j0 : INT32_MAX, b3 = valid ? -A.j0 : INT32_MAX;
    for (int o = 32; o >= 1; o >>= 1) {
        b0 = min(b0, __shfl_xor(b0, o));
        b1 = min(b1, __shfl_xor(b1, o));
        b2 = min(b2, __shfl_xor(b2, o));
        b3 = min(b3, __shfl_xor(b3, o));
    }
    if (lane == 0) {
        s_red[wave][0] = b0;
        s_red[wave][1] = b1;
        s_red[wave][2] = b2;
        s_red[wave][3] = b3;
    }
    s_fi[t] = A.i0;
    s_fj[t] = A.j0;
    s_ffx[t] = A.fx;
    s_ffy[t] = A.fy;
    s_fzb[t] = A.zb;
    __syncthreads();
    for (int w = 0; w < kRpcfT / 64; ++w) {
        b0 = min(b0, s_red[w][0]);
        b1 = min(b1, s_red[w][1]);
        b2 = min(b2, s_red[w][2]);
        b3 = min(b3, s_red[w][3]);
    }
    if (b0 == INT32_MAX) return;  // no fragment in this tile (uniform)
    const int nbc = 2 * r + 3;    // bits of a column word
    const int fw = (-b1) - b0, fh = (-b3) - b2;  // texel box extent - 1
    const int hx = b0 - R, hy = b2 - r - 1;
    const int hw = fw + 2 * R + 1, hh = fh + 2 * r + 3;
    // column words read 8 texels at a time: up to 7 more rows; an odd column
    // length keeps the transposing stores conflict-free
    const int vx = b0 - r - 1, vy = b2 - R;
    const int vwd = fw + 2 * r + 3, vh = (fh + 2 * R + 1 + 7) | 1;
    const int hrows = VB ? hh : hh + 7;  // without V, column words read whole chunks of 8 rows of H
    const bool staged = (int64_t)hw * hrows + (VB ? (int64_t)vwd * vh : 0) <= cap;
    float *hb = s_band, *vb = s_band + (staged ? hw * hrows : 0);
    if (staged) {
        {
            const int area = hw * hrows;
            int y = t / hw, x = t % hw;
            const int dy = kRpcfT / hw, dx = kRpcfT % hw;
            for (int idx = t; idx < area; idx += kRpcfT) {
                hb[idx] = canon(texel(m, hx + x, hy + y));
                y += dy;
                x += dx;
                if (x >= hw) {
                    x -= hw;
                    ++y;
                }
            }
        }
        if (VB) {
            // read row by row (coalesced), store transposed
            const int area = vwd * vh;
            int y = t / vwd, x = t % vwd;
            const int dy = kRpcfT / vwd, dx = kRpcfT % vwd;
            for (int idx = t; idx < area; idx += kRpcfT) {
                vb[x * vh + y] = canon(texel(m, vx + x, vy + y));
                y += dy;
                x += dx;
                if (x >= vwd) {
                    x -= vwd;
                    ++y;
                }
            }
        }
    }
    __syncthreads();
    const lds_float *hbl = (const lds_float *)hb, *vbl = (const lds_float *)vb;

    // shadow-test bits of column i, rows j0-r-1 .. j0+r+1
    auto colword = [&](int i) -> uint64_t {
        if (!valid) return 0ull;
        if (staged) {
            if constexpr (VB) {
                const lds_float *line = vbl + (i - vx) * vh + (A.j0 - r - 1 - vy);
                return shadow_bits([&](int q) { return line[q]; }, nbc, A.zb);
            } else {
                const lds_float *col = hbl + (A.j0 - r - 1 - hy) * hw + (i - hx);
                return shadow_bits([&](int q) { return col[q * hw]; }, nbc, A.zb);
            }
        }
        const int j = A.j0 - r - 1;
        return shadow_bits([&](int q) { return canon(texel(m, i, j + q)); }, nbc, A.zb);
    };

    const uint64_t range = ((1ull << (2 * r + 1)) - 1ull) << 1;  // rows j0-r .. j0+r
    double acc = 0.0;
    // two columns per round, a and a + 1: words cm (a-1), c0 (a), c1 (a+1), c2 (a+2)
    uint64_t cm = colword(A.i0 - r - 1), c0 = colword(A.i0 - r);
    for (int a = -r; a <= r; a += 2) {
        const bool two = a + 1 <= r;  // uniform
        const uint64_t c1 = colword(A.i0 + a + 1);
        const uint64_t c2 = two ? colword(A.i0 + a + 2) : 0ull;
        // discontinuity masks of column x (words w_-, w, w_+): L, R, T, B
        const uint64_t e0 = valid ? ((c0 ^ cm) | (c0 ^ c1) | (c0 ^ (c0 >> 1)) | (c0 ^ (c0 << 1))) & range : 0ull;
        const uint64_t e1 =
            valid && two ? ((c1 ^ c0) | (c1 ^ c2) | (c1 ^ (c1 >> 1)) | (c1 ^ (c1 << 1))) & range : 0ull;
        // terms without a discontinuity: their own test (lit = 1)
        acc += (double)__builtin_popcountll(~e0 & ~c0 & range);
        if (two) acc += (double)__builtin_popcountll(~e1 & ~c1 & range);

        // this round's terms with a discontinuity: offsets over the workgroup
        const int n0 = __builtin_popcountll(e0), ne = n0 + __builtin_popcountll(e1);
        int inc = ne;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        const int par = ((a + r) >> 1) & 1;  // double buffer: no barrier between rounds without such terms
        if (lane == 63) s_wtot[par][wave] = inc;
        // the previous round's readers of s_cw all passed its last barrier
        s_cw[0][t] = cm;
        s_cw[1][t] = c0;
        s_cw[2][t] = c1;
        s_cw[3][t] = c2;
        __syncthreads();
        int off = inc - ne, tot = 0;
        for (int w = 0; w < kRpcfT / 64; ++w) {
            const int x = s_wtot[par][w];
            off += w < wave ? x : 0;
            tot += x;
        }
        for (int w0 = 0; w0 < tot; w0 += kRpcfEnt) {  // uniform
            const int cnt = min(kRpcfEnt, tot - w0);
            // list this lane's terms that fall in [w0, w0 + cnt): column a, then a + 1
            if (off < w0 + cnt && off + ne > w0) {
                int e = off;
                for (int x = 0; x < 2; ++x) {
                    const uint64_t wl = x ? c0 : cm, w = x ? c1 : c0, wr = x ? c2 : c1;
                    uint64_t bits = x ? e1 : e0;
                    for (; bits; ++e) {
                        const int q = __builtin_ctzll(bits);
                        bits &= bits - 1ull;
                        if (e < w0 || e >= w0 + cnt) continue;
                        const uint32_t mk = (uint32_t)(((w ^ wl) >> q) & 1ull) * BIT_L |
                                            (uint32_t)(((w ^ wr) >> q) & 1ull) * BIT_R |
                                            (uint32_t)(((w ^ (w >> 1)) >> q) & 1ull) * BIT_T |
                                            (uint32_t)(((w ^ (w << 1)) >> q) & 1ull) * BIT_B;
                        const uint32_t lit_ = ((w >> q) & 1ull) == 0ull ? 1u : 0u;
                        s_ent[e - w0] = (uint32_t)t | (uint32_t)q << LB | lit_ << (LB + 6) | mk << (LB + 7) |
                                        (uint32_t)x << (LB + 11);
                    }
                }
            }
            __syncthreads();
            // one lane per term: its four traversals, normalization (Eq. 5) and Listing 5
            for (int e = t; e < cnt; e += kRpcfT) {
                const uint32_t en = s_ent[e];
                const int L = en & ((1u << LB) - 1u), q = (en >> LB) & 63;
                const bool s = (en >> (LB + 6)) & 1u;
                const unsigned mk = (en >> (LB + 7)) & 15u;
                const int i = s_fi[L] + a + (int)((en >> (LB + 11)) & 1u), j = s_fj[L] - r - 1 + q;
                const float zb = s_fzb[L];
                int rd[4];  // left, right, top, bottom
                if (staged) {
                    // H: rows j, j+1 (top), j-1 (bottom) along columns;
                    // V: columns i, i-1 (left), i+1 (right) along rows
                    // (without V: H down column i, the side columns at -+1)
                    const lds_float *ph = hbl + (j - hy) * hw;
                    const lds_float *pv = VB ? vbl + (i - vx) * vh : hbl + (i - hx);
                    const int vside = VB ? vh : 1;
                    BandWalkReader bh, bv;
                    bh.c = (lds_byte *)ph;
                    bh.a = (lds_byte *)(ph + hw);
                    bh.b = (lds_byte *)(ph - hw);
                    bh.step = 4u;
                    bv.c = (lds_byte *)pv;
                    bv.a = (lds_byte *)(pv - vside);
                    bv.b = (lds_byte *)(pv + vside);
                    bv.step = VB ? 4u : 4u * (unsigned)hw;
                    const int ph0 = i - hx, pv0 = VB ? j - vy : j - hy;
                    const int vlen = VB ? vh : hrows;  // band positions of a vertical traversal
                    const bool ht = (mk & BIT_T) != 0, hbt = (mk & BIT_B) != 0;
                    const bool vl = (mk & BIT_L) != 0, vr = (mk & BIT_R) != 0;
                    // the fragment's column words of the term's column and its
                    // neighbours (rows j0-r-1 .. j0+r+1): the horizontal
                    // traversals' first steps, and the vertical ones as far
                    // as the words reach
                    const int x = (en >> (LB + 11)) & 1u;
                    const uint64_t wl = s_cw[x][L], w = s_cw[x + 1][L], wr = s_cw[x + 2][L];
                    rd[0] = first_steps(bh, wl, q, ph0, -1, maxd, zb, s, ht, hbt);
                    rd[1] = first_steps(bh, wr, q, ph0, 1, maxd, zb, s, ht, hbt);
                    int k0[4] = {3, 3, 0, 0};
                    rd[2] = column_walk_up(wl, w, wr, q, nbc, maxd, s, vl, vr, k0[2]);
                    rd[3] = column_walk_down(wl, w, wr, q, maxd, s, vl, vr, k0[3]);
                    // the few that run on
                    for (int dir = 0; dir < 4; ++dir) {
                        if (rd[dir] != 0) continue;
                        const bool horiz = dir < 2;
                        const int d = dir == 0 || dir == 3 ? -1 : 1;
                        const int p0 = horiz ? ph0 : pv0;
                        const bool ca = horiz ? ht : vl, cb = horiz ? hbt : vr;
                        // last step inside the band
                        const int kl = min(maxd, d > 0 ? (horiz ? hw : vlen) - 1 - p0 : p0);
                        int x = 0;
                        if (k0[dir] <= kl)
                            x = walk_range<4>(horiz ? bh : bv, k0[dir], kl, p0, d, INT32_MAX / 4, zb, s, ca, cb);
                        if (x == 0 && kl < maxd) {
                            const MapLineReader g{m, horiz ? j : i, horiz ? j + 1 : i - 1, horiz ? j - 1 : i + 1,
                                                  horiz};
                            x = walk_range<4>(g, max(k0[dir], kl + 1), maxd, horiz ? i : j, d,
                                              horiz ? m.W - 1 : m.H - 1, zb, s, ca, cb);
                        }
                        rd[dir] = x != 0 ? x : -(maxd + 1);
                    }
                } else {
                    rd[0] = walk_dir(m, i, j, zb, s, mk, maxd, -1, 0);
                    rd[1] = walk_dir(m, i, j, zb, s, mk, maxd, 1, 0);
                    rd[2] = walk_dir(m, i, j, zb, s, mk, maxd, 0, 1);
                    rd[3] = walk_dir(m, i, j, zb, s, mk, maxd, 0, -1);
                }
                const Axis axx = normalize_axis(rd[0], rd[1], s_ffx[L]);
                const Axis axy = normalize_axis(rd[3], rd[2], s_ffy[L]);
                s_val[e] = vis_rsmss(s, axx, axy);
            }
            __syncthreads();
            // each fragment adds its own terms, in list order
            const int e_lo = max(off, w0), e_hi = min(off + ne, w0 + cnt);
            for (int e = e_lo; e < e_hi; ++e) acc += (double)s_val[e - w0];
        }
        cm = c1;
        c0 = c2;
    }
    if (valid) out[k] = (float)(acc / (double)((2 * r + 1) * (2 * r + 1)));
}

// Radii up to this one stage the transposed band V (faster column words);
// larger ones only H (half the LDS, more workgroups per CU).  Measured on the
// 4K fenced frame, with V / without: r = 5 1.19 / 1.46 ms, 9 3.77 / 4.28,
// 10 4.98 / 4.89, 13 8.43 / 7.25, 15 10.5 / 9.23 (before the kernel was held
// to 128 VGPRs, which brought the H-only form to 4.32 / 6.38 / 8.78 ms at
// r = 10 / 13 / 15).
constexpr int kRpcfTransposedMaxR = 9;

// LDS texels for the staged bands of an RPCF workgroup: enough for a tile
// whose texel footprint spans up to 13 x 17 texels, within 64 KiB with the
// kernel's static LDS.
inline int rpcf_cap(int r, int maxd) {
    const int R = r + (maxd < kRpcfReach ? maxd : kRpcfReach);
    const int want = r <= kRpcfTransposedMaxR
                         ? (12 + 2 * R + 1) * (16 + 2 * r + 3) + (12 + 2 * r + 3) * ((16 + 2 * R + 1 + 7) | 1)
                         : (12 + 2 * R + 1) * (16 + 2 * r + 3 + 7);
    const int room = (65536 - 12288) / 4;
    return want < room ? want : room;
}

inline void launch_rpcf(const MapView &mv, const float *frags, int64_t n, int64_t view_width, float bias, int maxd,
                        int r, float *out, hipStream_t stream) {
    if (r > kRpcfMaxR) {
        hipLaunchKernelGGL(rpcf_naive_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, mv, frags,
                           n, bias, maxd, r, out);
        return;
    }
    const int cap = rpcf_cap(r, maxd);
    const size_t lds = (size_t)cap * 4;
    if (view_width > 0) {
        constexpr int TW = 16, TH = kRpcfT / TW;
        const int64_t rows = (n + view_width - 1) / view_width;
        const int64_t tiles_x = (view_width + TW - 1) / TW;
        const int64_t tiles = tiles_x * ((rows + TH - 1) / TH);
        if (r <= kRpcfTransposedMaxR)
            hipLaunchKernelGGL((rpcf_kernel<TW, true>), dim3((unsigned)tiles), dim3(kRpcfT), lds, stream, mv, frags,
                               n, view_width, tiles_x, bias, maxd, r, cap, out);
        else
            hipLaunchKernelGGL((rpcf_kernel<TW, false>), dim3((unsigned)tiles), dim3(kRpcfT), lds, stream, mv, frags,
                               n, view_width, tiles_x, bias, maxd, r, cap, out);
    } else {
        const int64_t tiles = (n + kRpcfT - 1) / kRpcfT;
        if (r <= kRpcfTransposedMaxR)
            hipLaunchKernelGGL((rpcf_kernel<kRpcfT, true>), dim3((unsigned)tiles), dim3(kRpcfT), lds, stream, mv,
                               frags, n, n, tiles, bias, maxd, r, cap, out);
        else
            hipLaunchKernelGGL((rpcf_kernel<kRpcfT, false>), dim3((unsigned)tiles), dim3(kRpcfT), lds, stream, mv,
                               frags, n, n, tiles, bias, maxd, r, cap, out);
    }
}

}  // namespace rbsm
