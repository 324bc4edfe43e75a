/*
 * CPU oracle for revectorization-based shadow mapping (RBSM): hard silhouette
 * recovery and the filtered variant (RSMSS), from Macedo, Apolinario, Aguero,
 * "Optimized Visibility Functions for Revectorization-Based Shadow Mapping"
 * (arXiv 1711.07793).
 *
 * TEST INFRASTRUCTURE.  This file is the slow, plain reference the GPU path is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product library never does.  It shares no
 * code, header or constant with the GPU path.
 *
 * Precision: the paper's listings compute in GLSL float, so the oracle computes
 * in IEEE binary32 in the order the listings write, built without FMA
 * contraction (-ffp-contract=off) and without -ffast-math.  Binary64 appears
 * only in the decision-margin helper used to confirm that a disagreement sits
 * on a decision boundary.
 *
 * Readings of points the paper leaves open (each also recorded in the design
 * notes):
 *  - nearest-texel addressing: X = u*W, texel floor(X), sub-texel fraction
 *    X - floor(X); every texel index is clamped to the map (clamp-to-edge);
 *  - the depth test is Eq. 1 with a caller bias: lit unless (z - bias) > T,
 *    with z - bias rounded to binary32 once;
 *  - neighbour and traversal steps move by whole texels;
 *  - checkDiscontinuity (called but not defined in the traversal listing) is
 *    true when the visited texel, tested at the fragment's own depth, has a
 *    discontinuity in at least one direction in which the fragment has one
 *    (Sec. 3.1.3, "share at least one discontinuity direction");
 *  - computeFragmentDistanceToSE walks left, right, top (+y), bottom (-y);
 *  - normalizeFragmentDistanceToSE: per axis, count the walks that found an
 *    end (Eq. 5 code: 2 -> 1, 1 -> 0, 0 -> -1).  With one end, the
 *    normalized distance is the distance from the fragment to the boundary of
 *    the end texel divided by the number of edge texels on that axis
 *    (|rd-| + |rd+| - 1); with no end it is 1, with two ends 0;
 *  - the RSMSS I-shape test reads nrd.w == -1 (the printed "nrd.w == 1.0" is
 *    unreachable there);
 *  - RPCF (radius r > 0): box average of the RSMSS value evaluated at the
 *    (2r+1)^2 texels around the fragment's texel with the same sub-texel
 *    position and depth (Sec. 5.3 suggests PCF to suppress skeleton artifacts).
 *    The paper fixes no summation order or precision.  The result is defined
 *    as the exact mean of the (2r+1)^2 binary32 terms rounded to binary32;
 *    the oracle approximates that mean by summing the terms in binary64 in
 *    row-major offset order (a outer, b inner), dividing once in binary64 and
 *    rounding to binary32.  For M = (2r+1)^2 <= 4225 terms in [0, 1] the
 *    binary64 sum is within (M - 1) M 2^-53 < 2e-9 of the exact sum in any
 *    order, so any binary64 evaluation order lands within 5e-13 of the exact
 *    mean before the final rounding: two orders give equal or adjacent
 *    binary32 results.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t width, height;
    int64_t pitch;
    float depth_bias;
    int32_t max_dist;
    int32_t kernel_radius;
} oracle_params;

/* Optional instrumentation: when non-null every texel read is marked here
 * (row-major, width*height bytes) and counted. */
static uint8_t *g_touch = NULL;
static int64_t g_fetches = 0;

void oracle_set_touch(uint8_t *touch) {
    g_touch = touch;
    g_fetches = 0;
}
int64_t oracle_fetch_count(void) { return g_fetches; }

/* texture2D(SM, ...).z with nearest filtering and clamp-to-edge */
static float fetch(const float *map, const oracle_params *p, int i, int j) {
    if (i < 0) i = 0;
    if (i > p->width - 1) i = p->width - 1;
    if (j < 0) j = 0;
    if (j > p->height - 1) j = p->height - 1;
    if (g_touch) {
        g_touch[(int64_t)j * p->width + i] = 1;
        ++g_fetches;
    }
    return map[(int64_t)j * p->pitch + i];
}

/* Eq. 1: s = 0 if p_z > z(t), 1 otherwise (pz already carries the bias). */
static float shadow_test(float pz, float blocker) { return pz > blocker ? 0.0f : 1.0f; }

/* Eq. 2-3: the neighbour tests at the fragment's own depth and the
 * discontinuity directions they give.  Bit L (1), R (2), T (4, +y) or B
 * (8, -y) is set when that 4-connected neighbour's test differs from the
 * texel's own test s. */
enum { DIR_L = 1, DIR_R = 2, DIR_T = 4, DIR_B = 8 };

static unsigned discontinuity_dirs(const float *map, const oracle_params *p, int i, int j, float pz,
                                   float s) {
    unsigned bits = 0;
    if (shadow_test(pz, fetch(map, p, i - 1, j)) != s) bits |= DIR_L;
    if (shadow_test(pz, fetch(map, p, i + 1, j)) != s) bits |= DIR_R;
    if (shadow_test(pz, fetch(map, p, i, j + 1)) != s) bits |= DIR_T;
    if (shadow_test(pz, fetch(map, p, i, j - 1)) != s) bits |= DIR_B;
    return bits;
}

/* Eq. 4: the compressed discontinuity vector of Table 1,
 * d = ((2 dL + dR) / 4, (2 dT + dB) / 4, 1 - s). */
static void compress_discontinuity(unsigned bits, float s, float d[3]) {
    const float dl = (bits & DIR_L) ? 1.0f : 0.0f, dr = (bits & DIR_R) ? 1.0f : 0.0f;
    const float dt = (bits & DIR_T) ? 1.0f : 0.0f, db = (bits & DIR_B) ? 1.0f : 0.0f;
    d[0] = (2.0f * dl + dr) / 4.0f;
    d[1] = (2.0f * dt + db) / 4.0f;
    d[2] = 1.0f - s;
}

/* Sec. 3.1.3: the distance from the fragment's texel to the end of its
 * shadow edge in direction (dx, dy).  Texel k = 1, 2, ... max_dist along the
 * direction either has the opposite test (the edge ends there: +k), or no
 * longer shares a discontinuity direction with the fragment's texel (the
 * edge leaves the direction without ending: -k); if neither happens within
 * max_dist texels the edge is taken as unbounded, -(max_dist + 1). */
static int edge_distance(const float *map, const oracle_params *p, int i0, int j0, float pz, float s,
                         unsigned dirs0, int dx, int dy) {
    for (int k = 1; k <= p->max_dist; ++k) {
        const int i = i0 + k * dx, j = j0 + k * dy;
        if (shadow_test(pz, fetch(map, p, i, j)) != s) return k;
        if ((discontinuity_dirs(map, p, i, j, pz, s) & dirs0) == 0) return -k;
    }
    return -(p->max_dist + 1);
}

/* Sec. 3.1.4 and Eq. 5: one axis of the normalized discontinuity space,
 * from the walks toward its negative and positive side.  The code counts the
 * walks that found an end (two -> 1, one -> 0, none -> -1).  With exactly one
 * end the coordinate is the fragment's distance to the boundary of the end
 * texel over the number of edge texels on the axis; an axis without an end
 * reads 1 and one with two ends 0 (that value is never used). */
static void normalize_axis(int rd_neg, int rd_pos, float f, float *nrd, float *code) {
    const int ends = (rd_neg > 0) + (rd_pos > 0);
    if (ends == 2) {
        *code = 1.0f;
        *nrd = 0.0f;
    } else if (ends == 0) {
        *code = -1.0f;
        *nrd = 1.0f;
    } else {
        *code = 0.0f;
        const int an = rd_neg < 0 ? -rd_neg : rd_neg;
        const int ap = rd_pos < 0 ? -rd_pos : rd_pos;
        const float len = (float)(an + ap - 1);
        const float a = rd_pos > 0 ? (float)rd_pos - f : (float)(an - 1) + f;
        *nrd = a / len;
    }
}

/* Shape of the shadow edge at the fragment (Fig. 3; Sec. 3.1.4), read off
 * each axis separately.  An axis is closed when the edge ends on both of its
 * sides: either both neighbours on the axis already have the opposite test
 * (d == 0.75, the short shapes of Sec. 4) or both walks along it found an
 * end (code 1).  It is open when no walk along it found an end (code -1).
 *   both axes closed               -> O
 *   one axis closed                -> U (a ramp along the other axis)
 *   otherwise, an open axis        -> I (a straight edge)
 *   otherwise (one end per axis)   -> L (clipped by the revectorized edge) */
typedef enum { SHAPE_O, SHAPE_U_ALONG_Y, SHAPE_U_ALONG_X, SHAPE_I, SHAPE_L } edge_shape;

static edge_shape classify_shape(const float d[3], const float nrd[4]) {
    const int x_closed = d[0] == 0.75f || nrd[2] == 1.0f;
    const int y_closed = d[1] == 0.75f || nrd[3] == 1.0f;
    if (x_closed && y_closed) return SHAPE_O;
    if (x_closed) return SHAPE_U_ALONG_Y;
    if (y_closed) return SHAPE_U_ALONG_X;
    if (nrd[2] == -1.0f || nrd[3] == -1.0f) return SHAPE_I;
    return SHAPE_L;
}

static float clamp01(float x) {
    const float lo = x > 0.0f ? x : 0.0f;
    return lo < 1.0f ? lo : 1.0f;
}

/* Silhouette recovery (Sec. 3.1.4; the optimized function of Sec. 4) for a
 * lit fragment on an edge: closed shapes are put in shadow, straight edges
 * stay lit, and an L shape is shadowed below the revectorized edge, the line
 * nrd.y = 1 - nrd.x (a point on the line stays lit). */
static float hard_visibility(edge_shape shape, const float nrd[4]) {
    switch (shape) {
        case SHAPE_O:
        case SHAPE_U_ALONG_X:
        case SHAPE_U_ALONG_Y:
            return 0.0f;
        case SHAPE_I:
            return 1.0f;
        default:
            return nrd[1] < 1.0f - nrd[0] ? 0.0f : 1.0f;
    }
}

/* Revectorization-based filtering (Sec. 3.2; the optimized function of
 * Sec. 4) for a fragment on an edge, lit or shadowed (d.z = 1 - s).  With
 * sg = 1 - 2 d.z the value moves away from d.z by the normalized distances:
 * an O shape keeps d.z, a U shape ramps along its open axis, a straight edge
 * returns the test itself (1 - d.z), and an L shape adds both ramps, in the
 * order y then x, clamped to [0, 1]. */
static float filtered_visibility(edge_shape shape, const float d[3], const float nrd[4]) {
    const float dz = d[2];
    const float sg = 1.0f - 2.0f * dz;
    switch (shape) {
        case SHAPE_O:
            return dz;
        case SHAPE_U_ALONG_Y:
            return dz + sg * nrd[1];
        case SHAPE_U_ALONG_X:
            return dz + sg * nrd[0];
        case SHAPE_I:
            return 1.0f - dz;
        default: {
            const float along_y = dz + sg * nrd[1];
            return clamp01(along_y + sg * nrd[0]);
        }
    }
}

/* Everything the pass computes for one fragment at texel (i0, j0). */
typedef struct {
    float s;        /* centre test */
    float d[3];     /* compressed discontinuity */
    int32_t rd[4];  /* left, right, top, bottom; 0 when not traversed */
    float nrd[4];   /* normalized distances (x, y) and codes (z, w) */
    int32_t path;   /* 0 early shadow exit (hard), 1 no discontinuity, 2 revectorized */
    float vis;
} oracle_detail;

/* The RBSM listing for one fragment whose texel is (i0, j0), sub-texel
 * position (fx, fy), depth pz (bias applied). hard != 0 selects silhouette
 * recovery, else filtering. */
static void rbsm_at(const float *map, const oracle_params *p, int i0, int j0, float fx, float fy,
                    float pz, int hard, oracle_detail *out) {
    memset(out, 0, sizeof(*out));
    /* Eq. 1 at the fragment's texel; silhouette recovery only ever works on
     * the lit side, so a shadowed fragment stays shadowed */
    const float s = shadow_test(pz, fetch(map, p, i0, j0));
    out->s = s;
    if (hard && s == 0.0f) {
        out->path = 0;
        out->vis = s;
        return;
    }
    /* Eq. 2-4: no discontinuity means no shadow edge: the plain test */
    const unsigned dirs0 = discontinuity_dirs(map, p, i0, j0, pz, s);
    compress_discontinuity(dirs0, s, out->d);
    if (dirs0 == 0) {
        out->path = 1;
        out->vis = s;
        return;
    }
    /* Sec. 3.1.3: distances to the edge ends, left, right, top, bottom */
    const int step[4][2] = {{-1, 0}, {+1, 0}, {0, +1}, {0, -1}};
    for (int w = 0; w < 4; ++w) out->rd[w] = edge_distance(map, p, i0, j0, pz, s, dirs0, step[w][0], step[w][1]);
    /* Eq. 5: x from (left, right) and fx, y from (bottom, top) and fy */
    normalize_axis(out->rd[0], out->rd[1], fx, &out->nrd[0], &out->nrd[2]);
    normalize_axis(out->rd[3], out->rd[2], fy, &out->nrd[1], &out->nrd[3]);
    out->path = 2;
    const edge_shape shape = classify_shape(out->d, out->nrd);
    out->vis = hard ? hard_visibility(shape, out->nrd) : filtered_visibility(shape, out->d, out->nrd);
}

/* Fragment addressing: texel and sub-texel fraction from (u, v). */
static void address(const oracle_params *p, const float *frag, int *i0, int *j0, float *fx,
                    float *fy, float *pz) {
    const float X = frag[0] * (float)p->width;
    const float Y = frag[1] * (float)p->height;
    const float flx = floorf(X), fly = floorf(Y);
    *i0 = (int)flx;
    *j0 = (int)fly;
    *fx = X - flx;
    *fy = Y - fly;
    *pz = frag[2] - p->depth_bias;
}

static int params_ok(const oracle_params *p) {
    return p && p->width >= 1 && p->height >= 1 && p->pitch >= p->width && p->max_dist >= 1 &&
           p->kernel_radius >= 0;
}

/* Fragments must be finite with |u*W|, |v*H| < 2^20 (the oracle does not
 * extend addressing beyond that range). */
static int frag_ok(const oracle_params *p, const float *f) {
    if (!isfinite(f[0]) || !isfinite(f[1]) || !isfinite(f[2])) return 0;
    return fabsf(f[0] * (float)p->width) < 1048576.0f && fabsf(f[1] * (float)p->height) < 1048576.0f;
}

/* Plain shadow mapping (Eq. 1 only). out: 0 shadow, 1 lit. */
int oracle_shadow_map(const float *map, const float *frags, int64_t n, const oracle_params *p,
                      uint8_t *out) {
    if (!params_ok(p)) return -1;
    for (int64_t k = 0; k < n; ++k) {
        const float *f = frags + 3 * k;
        if (!frag_ok(p, f)) return -2;
        int i0, j0;
        float fx, fy, pz;
        address(p, f, &i0, &j0, &fx, &fy, &pz);
        out[k] = (uint8_t)shadow_test(pz, fetch(map, p, i0, j0));
    }
    return 0;
}

/* Hard RBSM (silhouette recovery). out: 0 shadow, 1 lit. */
int oracle_rbsm_hard(const float *map, const float *frags, int64_t n, const oracle_params *p,
                     uint8_t *out) {
    if (!params_ok(p) || p->kernel_radius != 0) return -1;
    for (int64_t k = 0; k < n; ++k) {
        const float *f = frags + 3 * k;
        if (!frag_ok(p, f)) return -2;
        int i0, j0;
        float fx, fy, pz;
        address(p, f, &i0, &j0, &fx, &fy, &pz);
        oracle_detail det;
        rbsm_at(map, p, i0, j0, fx, fy, pz, 1, &det);
        out[k] = (uint8_t)det.vis;
    }
    return 0;
}

/* RSMSS (filtered); with kernel_radius r > 0, the RPCF box average. */
int oracle_rsmss(const float *map, const float *frags, int64_t n, const oracle_params *p,
                 float *out) {
    if (!params_ok(p)) return -1;
    const int r = p->kernel_radius;
    const double count = (double)((2 * r + 1) * (2 * r + 1));
    for (int64_t k = 0; k < n; ++k) {
        const float *f = frags + 3 * k;
        if (!frag_ok(p, f)) return -2;
        int i0, j0;
        float fx, fy, pz;
        address(p, f, &i0, &j0, &fx, &fy, &pz);
        oracle_detail det;
        if (r == 0) {
            rbsm_at(map, p, i0, j0, fx, fy, pz, 0, &det);
            out[k] = det.vis;
            continue;
        }
        double sum = 0.0;
        for (int a = -r; a <= r; ++a)
            for (int b = -r; b <= r; ++b) {
                rbsm_at(map, p, i0 + a, j0 + b, fx, fy, pz, 0, &det);
                sum += (double)det.vis;
            }
        out[k] = (float)(sum / count);
    }
    return 0;
}

/* Per-fragment intermediate values, for tests.  hard selects the variant. */
int oracle_detail_one(const float *map, const float *frag, const oracle_params *p, int hard,
                      oracle_detail *out) {
    if (!params_ok(p) || !frag_ok(p, frag)) return -1;
    int i0, j0;
    float fx, fy, pz;
    address(p, frag, &i0, &j0, &fx, &fy, &pz);
    rbsm_at(map, p, i0, j0, fx, fy, pz, hard, out);
    return 0;
}

/* Batched helper for tiny-map enumeration: fragment k reads map number
 * map_index[k] from a stack of equally sized maps (map_stride floats apart). */
int oracle_multi(const float *maps, int64_t map_stride, const int32_t *map_index,
                 const float *frags, int64_t n, const oracle_params *p, int hard, float *vis,
                 int32_t *rd_out, float *nrd_out) {
    if (!params_ok(p)) return -1;
    for (int64_t k = 0; k < n; ++k) {
        const float *f = frags + 3 * k;
        if (!frag_ok(p, f)) return -2;
        int i0, j0;
        float fx, fy, pz;
        address(p, f, &i0, &j0, &fx, &fy, &pz);
        oracle_detail det;
        rbsm_at(maps + (int64_t)map_index[k] * map_stride, p, i0, j0, fx, fy, pz, hard, &det);
        vis[k] = det.vis;
        if (rd_out) memcpy(rd_out + 4 * k, det.rd, sizeof(det.rd));
        if (nrd_out) memcpy(nrd_out + 4 * k, det.nrd, sizeof(det.nrd));
    }
    return 0;
}

/* Binary64 decision margin of one fragment: the smallest distance to a
 * decision boundary over every depth test the pass can perform for it (the
 * texels on the two axes through its texel within max_dist + 1, and their
 * side neighbours), and, for an L-shaped edge, over the revectorized-edge
 * test |nrd.y - (1 - nrd.x)| recomputed in binary64 from the same integer
 * walk.  Used only to confirm that a GPU/oracle disagreement of a hard mask
 * is a rounding tie. */
double oracle_margin_one(const float *map, const float *frag, const oracle_params *p, int hard) {
    if (!params_ok(p) || !frag_ok(p, frag)) return -1.0;
    int i0, j0;
    float fx, fy, pz;
    address(p, frag, &i0, &j0, &fx, &fy, &pz);
    const double X = (double)frag[0] * p->width, Y = (double)frag[1] * p->height;
    const double zb = (double)frag[2] - (double)p->depth_bias;
    /* depth margins over every texel the pass can read for this fragment */
    uint8_t *saved = g_touch;
    g_touch = NULL;
    oracle_detail det;
    rbsm_at(map, p, i0, j0, fx, fy, pz, hard, &det);
    double m = 1e300;
    const int reach = p->max_dist + 1;
    for (int dj = -reach; dj <= reach; ++dj)
        for (int di = -reach; di <= reach; ++di) {
            if (abs(di) > 1 && abs(dj) > 1) continue; /* walks run along the axes */
            const double t = fetch(map, p, i0 + di, j0 + dj);
            const double g = fabs(zb - t);
            if (g < m) m = g;
        }
    if (det.path == 2 && det.nrd[2] == 0.0f && det.nrd[3] == 0.0f) {
        const double ffx = X - floor(X), ffy = Y - floor(Y);
        double nx, ny;
        {
            const int an = abs(det.rd[0]), ap = abs(det.rd[1]);
            const double len = an + ap - 1;
            nx = (det.rd[1] > 0 ? ap - ffx : (an - 1) + ffx) / len;
        }
        {
            const int an = abs(det.rd[3]), ap = abs(det.rd[2]);
            const double len = an + ap - 1;
            ny = (det.rd[2] > 0 ? ap - ffy : (an - 1) + ffy) / len;
        }
        const double g = fabs(ny - (1.0 - nx));
        if (g < m) m = g;
    }
    g_touch = saved;
    return m;
}

/* Multi-light compositing (serving extension): the per-fragment weighted sum
 * of per-light visibilities, out[k] = sum over lights in order of
 * weights[l] * vis_l[k], each product rounded to binary32, then added.  The
 * visibility scales one light's contribution (Listing 1); how lights combine
 * is not in the paper, so the weights are per-light intensities.  vis[l] is a
 * uint8 mask (hard[l] != 0) or a float visibility. */
int oracle_composite(int64_t n, int n_lights, const void *const *vis, const int32_t *hard, const float *weights,
                     float *out) {
    if (n < 0 || n_lights < 1 || n_lights > 8) return -1;
    for (int64_t k = 0; k < n; ++k) {
        float acc = 0.0f;
        for (int l = 0; l < n_lights; ++l) {
            float v;
            if (hard[l]) v = (float)((const uint8_t *)vis[l])[k];
            else v = ((const float *)vis[l])[k];
            const float term = weights[l] * v;
            acc = acc + term;
        }
        out[k] = acc;
    }
    return 0;
}

/* Shadow-map rasterization (on-device extension): the light pass producing
 * the depth map the shadow pass reads (Sec. 2 takes it as given).  A texel
 * samples its centre ((i + 0.5) / W, (j + 0.5) / H) and keeps the nearest
 * surface there: the receiver plane r0 + ru (u - .5) + rv (v - .5) (binary64,
 * rounded to binary32) or the depth of any primitive covering the centre,
 * whichever is smaller.  Polygons (convex, counter-clockwise) cover a point
 * when each edge's cross product (b - a) x (p - a) is positive, or zero on an
 * edge running downwards or horizontally to the left (top-left tie rule);
 * slabs cover o <= n.p < o + w.  Record layout: 112 bytes,
 * {int32 kind, int32 nv, double x[4], y[4], nx, ny, o, w, float depth, pad}. */
typedef struct {
    int32_t kind, nv;
    double x[4], y[4];
    double nx, ny, o, w;
    float depth;
    int32_t pad;
} oracle_prim;

static int prim_covers(const oracle_prim *q, double px, double py) {
    if (q->kind == 1) {
        const double t = q->nx * px + q->ny * py;
        return t >= q->o && t < q->o + q->w;
    }
    if (q->kind != 0 || q->nv < 3 || q->nv > 4) return 0;
    for (int a = 0; a < q->nv; ++a) {
        const int b = (a + 1) % q->nv;
        const double cross = (q->x[b] - q->x[a]) * (py - q->y[a]) - (q->y[b] - q->y[a]) * (px - q->x[a]);
        if (cross > 0.0) continue;
        if (cross < 0.0) return 0;
        const double dx = q->x[b] - q->x[a], dy = q->y[b] - q->y[a];
        const int owns = dy < 0.0 || (dy == 0.0 && dx < 0.0);
        if (!owns) return 0;
    }
    return 1;
}

int oracle_raster(const oracle_prim *prims, int n, double r0, double ru, double rv, int W, int H, int64_t pitch,
                  float *map) {
    if (n < 0 || W < 1 || H < 1 || pitch < W) return -1;
    for (int j = 0; j < H; ++j) {
        const double v = (j + 0.5) / H;
        for (int i = 0; i < W; ++i) {
            const double u = (i + 0.5) / W;
            float nearest = (float)(r0 + ru * (u - 0.5) + rv * (v - 0.5));
            for (int k = 0; k < n; ++k)
                if (prim_covers(&prims[k], u, v) && prims[k].depth < nearest) nearest = prims[k].depth;
            map[(int64_t)j * pitch + i] = nearest;
        }
    }
    return 0;
}

/* The same value at count chosen texels (i[k], j[k]) of a width x height map. */
int oracle_raster_texels(const oracle_prim *prims, int n, double r0, double ru, double rv, int W, int H,
                         const int32_t *ti, const int32_t *tj, int64_t count, float *out) {
    if (n < 0 || W < 1 || H < 1) return -1;
    for (int64_t k = 0; k < count; ++k) {
        if (ti[k] < 0 || ti[k] >= W || tj[k] < 0 || tj[k] >= H) return -2;
        const double u = (ti[k] + 0.5) / W, v = (tj[k] + 0.5) / H;
        float nearest = (float)(r0 + ru * (u - 0.5) + rv * (v - 0.5));
        for (int q = 0; q < n; ++q)
            if (prim_covers(&prims[q], u, v) && prims[q].depth < nearest) nearest = prims[q].depth;
        out[k] = nearest;
    }
    return 0;
}
