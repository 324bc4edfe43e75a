// RPCF: the RSMSS value averaged over the (2r+1)^2 texels around a
// fragment's texel, each evaluated with the fragment's own sub-texel position
// and depth (PCF over the filtered edge, Sec. 5.3).  Included once, by
// rbsm.hip.
//
// Every term of one fragment tests texels against the same depth, so the pass
// first turns the fragment's cross-shaped read region into shadow-test bits:
//   row words    rows j0-r-1 .. j0+r+1, columns i0-R .. i0+R (bit p <-> i0-R+p)
//   column words columns i0-r-1 .. i0+r+1, rows j0-R .. j0+R (bit q <-> j0-R+q)
// with R = r + MAXDIST, so a word holds a whole line a term's traversal can
// reach (2R+1 <= 63 bits).  A term's discontinuity mask is then a few shifts
// and XORs (Eq. 2-3); a term without a discontinuity contributes its test
// result, so those are counted with one popcount per column; and each bounded
// traversal of Listing 3 becomes one count of trailing (or leading) ones on
// "same test AND shares a discontinuity direction" bits (Sec. 3.1.3).  Only
// terms with a discontinuity run the normalization (Eq. 5) and Listing 5.
//
// The sum is kept in binary64 (exact for these terms in practice) and divided
// by (2r+1)^2 once, so the result is the box average rounded to binary32 once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbsm_device.hpp"
#include "tile_pass.hpp"

namespace rbsm {

constexpr int kRpcfT = 128;        // threads per workgroup, one fragment each
constexpr int kRpcfMaxReach = 31;  // largest r + MAXDIST whose lines fit one 64-bit word

// Any reach: one lane per fragment, every term evaluated from global memory
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
// t - zb.  For finite operands the difference is negative exactly when
// zb > t, except for t = -0, zb = +0 (difference -0, test lit); callers pass
// t + 0.0f, which turns -0 into +0.
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

// Bounded traversal towards increasing bit index from bit c.  `go` has a 1
// where a step may continue (same test as the term and a shared
// discontinuity direction), `same` where the test equals the term's.  The walk
// stops at the first k >= 1 whose bit is 0 in `go`: an end (+k) when that
// texel's test differs, else -k; -(maxd + 1) when it runs out.  Needs
// c + maxd <= 63.
__device__ __forceinline__ int walk_up_bits(uint64_t go, uint64_t same, int c, int maxd) {
    const int k = __builtin_ctzll(~(go >> (c + 1))) + 1;
    if (k > maxd) return -(maxd + 1);
    return ((same >> (c + k)) & 1ull) ? -k : k;
}

// The same towards decreasing bit index; needs 1 <= c and c - maxd >= 0.
__device__ __forceinline__ int walk_down_bits(uint64_t go, uint64_t same, int c, int maxd) {
    const int k = __builtin_clzll(~(go << (64 - c))) + 1;
    if (k > maxd) return -(maxd + 1);
    return ((same >> (c - k)) & 1ull) ? -k : k;
}

// One fragment's RPCF value from its row words (in LDS, word k of this lane
// at rows[k * kRpcfT]) and column words built one column ahead by col(i).
template <class ColFn>
__device__ __forceinline__ float rpcf_terms(const uint64_t *rows, ColFn col, const Addr &A, int r, int maxd) {
    const int R = r + maxd;
    const uint64_t range = ((1ull << (2 * r + 1)) - 1ull) << (R - r);
    double acc = 0.0;
    uint64_t cm = col(A.i0 - r - 1), c0 = col(A.i0 - r);
    for (int a = -r; a <= r; ++a) {
        const uint64_t cp = col(A.i0 + a + 1);
        const uint64_t Lc = c0 ^ cm, Rc = c0 ^ cp;
        const uint64_t Tc = c0 ^ (c0 >> 1), Bc = c0 ^ (c0 << 1);
        uint64_t edge = (Lc | Rc | Tc | Bc) & range;
        // terms without a discontinuity: their own test (lit = 1)
        acc += (double)__builtin_popcountll(~edge & ~c0 & range);
        while (edge) {
            const int q = __builtin_ctzll(edge);
            edge &= edge - 1ull;
            const bool s = ((c0 >> q) & 1ull) == 0ull;  // lit
            const bool bl = (Lc >> q) & 1ull, br = (Rc >> q) & 1ull;
            const bool bt = (Tc >> q) & 1ull, bb = (Bc >> q) & 1ull;
            // vertical traversals along the column word
            const uint64_t same_c = s ? ~c0 : c0;
            const uint64_t go_c = same_c & ((bl ? Lc : 0ull) | (br ? Rc : 0ull));
            const int rt = walk_up_bits(go_c, same_c, q, maxd);
            const int rb = walk_down_bits(go_c, same_c, q, maxd);
            // horizontal traversals along the term's row word
            const int kk = q - R + r + 1;
            const uint64_t h0 = rows[kk * kRpcfT];
            const uint64_t hp = rows[(kk + 1) * kRpcfT];
            const uint64_t hm = rows[(kk - 1) * kRpcfT];
            const int p = R + a;
            const uint64_t same_r = s ? ~h0 : h0;
            const uint64_t go_r = same_r & ((bt ? (h0 ^ hp) : 0ull) | (bb ? (h0 ^ hm) : 0ull));
            const int rr = walk_up_bits(go_r, same_r, p, maxd);
            const int rl = walk_down_bits(go_r, same_r, p, maxd);
            const Axis axx = normalize_axis(rl, rr, A.fx);
            const Axis axy = normalize_axis(rb, rt, A.fy);
            acc += (double)vis_rsmss(s, axx, axy);
        }
        cm = c0;
        c0 = cp;
    }
    return (float)(acc / (double)((2 * r + 1) * (2 * r + 1)));
}

// One workgroup per TW x (kRpcfT / TW) pixel tile of a row-major image of
// width vw (flat: vw = n, TW = kRpcfT).  When both fit in `cap` texels, the
// two bands the tile's words read are staged in LDS with clamped
// coordinates, -0 stored as +0: the fragments' texel box grown by R
// horizontally and r+1 vertically (row words), and grown by r+1 horizontally
// and R vertically, stored transposed (column words), each with up to 7 more
// texels along its lines for the 8-texel read chunks.  Every word is then
// built from contiguous LDS reads.  Otherwise the words are built from global
// memory.  Requires r >= 1, r + maxd <= kRpcfMaxReach.
template <int TW>
__global__ __launch_bounds__(kRpcfT) void rpcf_kernel(MapView m, const float *__restrict__ frags, int64_t n,
                                                      int64_t vw, int64_t tiles_x, float bias, int maxd, int r,
                                                      int cap, float *__restrict__ out) {
    extern __shared__ uint64_t s_rpcf[];  // row words [(2r+3)][kRpcfT], then the staged bands
    __shared__ int s_red[kRpcfT / 64][4];
    constexpr int TH = kRpcfT / TW;
    const int t = threadIdx.x;
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
    const int64_t px = txi * TW + (t % TW), py = tyi * TH + (t / TW);
    const int64_t k = py * vw + px;
    const bool valid = px < vw && k < n;
    Addr A{};
    if (valid) A = address(frags[3 * k + 0], frags[3 * k + 1], frags[3 * k + 2], m.W, m.H, bias);
    const int R = r + maxd;

    // texel box of the tile's fragments
    int b0 = valid ? A.i0 : INT32_MAX, b1 = valid ? -A.i0 : INT32_MAX;
    int b2 = valid ? A.j0 : INT32_MAX, b3 = valid ? -A.j0 : INT32_MAX;
    for (int o = 32; o >= 1; o >>= 1) {
        b0 = min(b0, __shfl_xor(b0, o));
        b1 = min(b1, __shfl_xor(b1, o));
        b2 = min(b2, __shfl_xor(b2, o));
        b3 = min(b3, __shfl_xor(b3, o));
    }
    if ((t & 63) == 0) {
        s_red[t >> 6][0] = b0;
        s_red[t >> 6][1] = b1;
        s_red[t >> 6][2] = b2;
        s_red[t >> 6][3] = b3;
    }
    __syncthreads();
    for (int w = 0; w < kRpcfT / 64; ++w) {
        b0 = min(b0, s_red[w][0]);
        b1 = min(b1, s_red[w][1]);
        b2 = min(b2, s_red[w][2]);
        b3 = min(b3, s_red[w][3]);
    }
    if (b0 == INT32_MAX) return;  // no fragment in this tile (uniform)
    const int nb = 2 * R + 1, pad = ((nb + 7) & ~7) - nb;
    const int fw = (-b1) - b0, fh = (-b3) - b2;  // texel box extent - 1
    // horizontal band (row words), row-major: rows b2-r-1 .. , columns b0-R ..
    const int hx = b0 - R, hy = b2 - r - 1;
    const int hw = fw + nb + pad, hh = fh + 2 * r + 3;
    // vertical band (column words), stored column by column: columns b0-r-1 ..,
    // rows b2-R .. ; an odd column length keeps the transposing stores
    // conflict-free
    const int vx = b0 - r - 1, vy = b2 - R;
    const int vw_ = fw + 2 * r + 3, vh = (fh + nb + pad) | 1;
    const bool staged = (int64_t)hw * hh + (int64_t)vw_ * vh <= cap;
    uint64_t *rows = s_rpcf + t;
    float *hb = reinterpret_cast<float *>(s_rpcf + (2 * r + 3) * kRpcfT);
    float *vb = hb + (staged ? hw * hh : 0);
    if (staged) {
        {
            const int area = hw * hh;
            int y = t / hw, x = t % hw;
            const int dy = kRpcfT / hw, dx = kRpcfT % hw;
            for (int idx = t; idx < area; idx += kRpcfT) {
                hb[idx] = texel(m, hx + x, hy + y) + 0.0f;
                y += dy;
                x += dx;
                if (x >= hw) {
                    x -= hw;
                    ++y;
                }
            }
        }
        {
            // read row by row (coalesced), store transposed
            const int area = vw_ * vh;
            int y = t / vw_, x = t % vw_;
            const int dy = kRpcfT / vw_, dx = kRpcfT % vw_;
            for (int idx = t; idx < area; idx += kRpcfT) {
                vb[x * vh + y] = texel(m, vx + x, vy + y) + 0.0f;
                y += dy;
                x += dx;
                if (x >= vw_) {
                    x -= vw_;
                    ++y;
                }
            }
        }
    }
    __syncthreads();
    if (!valid) return;

    float res;
    if (staged) {
        const float *row0 = hb + (A.j0 - r - 1 - hy) * hw + (A.i0 - R - hx);
        for (int kk = 0; kk < 2 * r + 3; ++kk) {
            const float *line = row0 + kk * hw;
            rows[kk * kRpcfT] = shadow_bits([&](int p) { return line[p]; }, nb, A.zb);
        }
        const int col0 = (A.j0 - R - vy) - vx * vh;
        res = rpcf_terms(
            rows,
            [&](int i) {
                const float *line = vb + (col0 + i * vh);
                return shadow_bits([&](int q) { return line[q]; }, nb, A.zb);
            },
            A, r, maxd);
    } else {
        for (int kk = 0; kk < 2 * r + 3; ++kk) {
            const int j = A.j0 - r - 1 + kk, i = A.i0 - R;
            rows[kk * kRpcfT] = shadow_bits([&](int p) { return texel(m, i + p, j) + 0.0f; }, nb, A.zb);
        }
        res = rpcf_terms(
            rows,
            [&](int i) {
                const int j = A.j0 - R;
                return shadow_bits([&](int q) { return texel(m, i, j + q) + 0.0f; }, nb, A.zb);
            },
            A, r, maxd);
    }
    out[k] = res;
}

// LDS texels for the staged bands of an RPCF workgroup: enough for a tile
// whose texel footprint spans up to 13 x 17 texels, within 64 KiB in all.
inline int rpcf_cap(int r, int maxd) {
    const int R = r + maxd;
    const int words = (2 * r + 3) * kRpcfT * 8;
    const int want = (12 + 2 * R + 8) * (16 + 2 * r + 3) + (12 + 2 * r + 3) * (16 + 2 * R + 9);
    const int room = (65536 - words - 256) / 4;
    return want < room ? want : room;
}

inline size_t rpcf_lds_bytes(int r, int cap) { return (size_t)(2 * r + 3) * kRpcfT * 8 + (size_t)cap * 4; }

inline void launch_rpcf(const MapView &mv, const float *frags, int64_t n, int64_t view_width, float bias, int maxd,
                        int r, float *out, hipStream_t stream) {
    if (r + maxd > kRpcfMaxReach) {
        hipLaunchKernelGGL(rpcf_naive_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, mv, frags,
                           n, bias, maxd, r, out);
        return;
    }
    const int cap = rpcf_cap(r, maxd);
    const size_t lds = rpcf_lds_bytes(r, cap);
    if (view_width > 0) {
        constexpr int TW = 16, TH = kRpcfT / TW;
        const int64_t rows = (n + view_width - 1) / view_width;
        const int64_t tiles_x = (view_width + TW - 1) / TW;
        const int64_t tiles = tiles_x * ((rows + TH - 1) / TH);
        hipLaunchKernelGGL((rpcf_kernel<TW>), dim3((unsigned)tiles), dim3(kRpcfT), lds, stream, mv, frags, n,
                           view_width, tiles_x, bias, maxd, r, cap, out);
    } else {
        const int64_t tiles = (n + kRpcfT - 1) / kRpcfT;
        hipLaunchKernelGGL((rpcf_kernel<kRpcfT>), dim3((unsigned)tiles), dim3(kRpcfT), lds, stream, mv, frags, n,
                           n, tiles, bias, maxd, r, cap, out);
    }
}

}  // namespace rbsm
