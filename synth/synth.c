/*
 * Seeded synthetic inputs for the revectorization-based shadow mapping pass.
 *
 * This module produces the two inputs of the per-fragment shadow pass: a
 * light-space depth map (the output of the light pass that the paper assumes
 * exists, Sec. 2 "Related Work", first paragraph) and camera fragments already
 * transformed into light space (the varying p of the RBSM listing, Sec. 3).
 * It holds none of the method's arithmetic: no shadow test, no neighbourhood
 * classification, no traversal, no visibility function.  Both the CPU oracle
 * and the GPU path consume its outputs.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) seeds xoshiro256**
 * (Blackman, Vigna, "Scrambled linear pseudorandom number generators",
 * ACM TOMS 2021).  Single floats are (x >> 40) * 2^-24, doubles
 * (x >> 11) * 2^-53, both uniform on [0, 1).
 *
 * Coordinates: u, v in [0, 1) address the map; texel (i, j) covers
 * [i/W, (i+1)/W) x [j/H, (j+1)/H) and is stored at map[j*pitch + i].  Depth
 * z grows away from the light; the receiver sits near 0.9, blockers in
 * [0.1, 0.8].  A texel is covered by a primitive iff its centre
 * ((i+.5)/W, (j+.5)/H) lies inside it (top-left rule on exact ties); its depth
 * is the minimum over covering primitives, else the receiver depth at the
 * texel centre.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYNTH_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* PRNG                                                                      */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t s[4]; } synth_rng;

static uint64_t splitmix64_next(uint64_t *state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

void synth_rng_seed(synth_rng *r, uint64_t seed) {
    uint64_t st = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64_next(&st);
}

uint64_t synth_rng_u64(synth_rng *r) {
    uint64_t *s = r->s;
    const uint64_t out = rotl64(s[1] * 5u, 7) * 9u;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return out;
}

static float rng_f32(synth_rng *r) { return (float)(synth_rng_u64(r) >> 40) * 0x1.0p-24f; }
static double rng_f64(synth_rng *r) { return (double)(synth_rng_u64(r) >> 11) * 0x1.0p-53; }
static double rng_range(synth_rng *r, double lo, double hi) { return lo + (hi - lo) * rng_f64(r); }
/* integer uniform on [lo, hi] inclusive */
static int rng_int(synth_rng *r, int lo, int hi) {
    return lo + (int)(rng_f64(r) * (double)(hi - lo + 1));
}

/* Fill out[n] with uniform floats in [0,1) (exposed for tests of the stream). */
void synth_uniform_f32(uint64_t seed, int64_t n, float *out) {
    synth_rng r;
    synth_rng_seed(&r, seed);
    for (int64_t k = 0; k < n; ++k) out[k] = rng_f32(&r);
}

/* ------------------------------------------------------------------------ */
/* Scenes                                                                    */
/* ------------------------------------------------------------------------ */

enum { PRIM_POLY = 0, PRIM_SLAB = 1 };

typedef struct {
    int kind;
    int nv;            /* PRIM_POLY: 3 or 4 vertices, counter-clockwise in (u, v) */
    double x[4], y[4];
    double nx, ny;     /* PRIM_SLAB: unit normal in (u, v) */
    double o, w;       /* PRIM_SLAB: covers o <= n.p < o + w */
    double depth;
} synth_prim;

typedef struct {
    int W, H;
    double r0, ru, rv; /* receiver depth r0 + ru (u - .5) + rv (v - .5) */
    int n;
    synth_prim *p;     /* sorted by increasing depth (closest to the light first) */
} synth_scene;

static double receiver_depth(const synth_scene *sc, double u, double v) {
    return sc->r0 + sc->ru * (u - 0.5) + sc->rv * (v - 0.5);
}

/* Edge function of directed edge a->b at point p: > 0 on the left (inside for CCW). */
static double edge_fn(double ax, double ay, double bx, double by, double px, double py) {
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

/* Top-left tie rule for a CCW polygon in a y-up frame: an exact tie on an edge
 * counts as inside when the edge runs downwards, or runs horizontally to the
 * left (the polygon's top edge). */
static int edge_owns_tie(double ax, double ay, double bx, double by) {
    const double dy = by - ay, dx = bx - ax;
    return (dy < 0.0) || (dy == 0.0 && dx < 0.0);
}

static int prim_contains(const synth_prim *q, double px, double py) {
    if (q->kind == PRIM_SLAB) {
        const double t = q->nx * px + q->ny * py;
        return t >= q->o && t < q->o + q->w;
    }
    for (int e = 0; e < q->nv; ++e) {
        const int f = (e + 1) % q->nv;
        const double val = edge_fn(q->x[e], q->y[e], q->x[f], q->y[f], px, py);
        if (val < 0.0) return 0;
        if (val == 0.0 && !edge_owns_tie(q->x[e], q->y[e], q->x[f], q->y[f])) return 0;
    }
    return 1;
}

static void make_ccw(synth_prim *q) {
    double a = 0.0;
    for (int e = 0; e < q->nv; ++e) {
        const int f = (e + 1) % q->nv;
        a += q->x[e] * q->y[f] - q->x[f] * q->y[e];
    }
    if (a < 0.0) {
        for (int e = 0; e < q->nv / 2; ++e) {
            const int f = q->nv - 1 - e;
            double t = q->x[e]; q->x[e] = q->x[f]; q->x[f] = t;
            t = q->y[e]; q->y[e] = q->y[f]; q->y[f] = t;
        }
    }
}

static int cmp_depth(const void *a, const void *b) {
    const double da = ((const synth_prim *)a)->depth, db = ((const synth_prim *)b)->depth;
    return (da > db) - (da < db);
}

void synth_scene_free(synth_scene *sc) {
    if (!sc) return;
    free(sc->p);
    free(sc);
}

static synth_scene *scene_alloc(int W, int H, int cap) {
    synth_scene *sc = (synth_scene *)calloc(1, sizeof(synth_scene));
    if (!sc) return NULL;
    sc->p = (synth_prim *)calloc((size_t)(cap > 0 ? cap : 1), sizeof(synth_prim));
    if (!sc->p) { free(sc); return NULL; }
    sc->W = W;
    sc->H = H;
    return sc;
}

/* One square blocker over a constant-depth receiver at 0.9: side U(0.3, 0.6)
 * of the map, rotation U[0, pi/2), centre U[0.3, 0.7]^2, depth U(0.2, 0.5). */
synth_scene *synth_scene_quad(uint64_t seed, int W, int H) {
    synth_scene *sc = scene_alloc(W, H, 1);
    if (!sc) return NULL;
    synth_rng r;
    synth_rng_seed(&r, seed);
    sc->r0 = 0.9; sc->ru = 0.0; sc->rv = 0.0;
    const double side = rng_range(&r, 0.3, 0.6);
    const double rot = rng_range(&r, 0.0, SYNTH_PI / 2.0);
    const double cx = rng_range(&r, 0.3, 0.7), cy = rng_range(&r, 0.3, 0.7);
    const double depth = rng_range(&r, 0.2, 0.5);
    synth_prim *q = &sc->p[0];
    q->kind = PRIM_POLY;
    q->nv = 4;
    const double c = cos(rot) * side * 0.5, s = sin(rot) * side * 0.5;
    const double ox[4] = {-1, 1, 1, -1}, oy[4] = {-1, -1, 1, 1};
    for (int k = 0; k < 4; ++k) {
        q->x[k] = cx + ox[k] * c - oy[k] * s;
        q->y[k] = cy + ox[k] * s + oy[k] * c;
    }
    make_ccw(q);
    q->depth = depth;
    sc->n = 1;
    return sc;
}

/* Random triangles over a tilted receiver 0.9 + 0.05 (u - .5) + 0.03 (v - .5):
 * vertex 0 uniform in [0,1]^2, two edges of log-uniform length in
 * [8, 512] texels at uniform angles (resampled until the triangle lies in
 * [0,1]^2), constant depth U(0.1, 0.8).  With fence != 0, add about 32
 * parallel bars 1-3 texels wide separated by 8-32 texel gaps at one random
 * angle and one depth U(0.1, 0.8). */
synth_scene *synth_scene_tris(uint64_t seed, int W, int H, int n_tris, int fence) {
    const int n_bars = fence ? 32 : 0;
    synth_scene *sc = scene_alloc(W, H, n_tris + n_bars);
    if (!sc) return NULL;
    synth_rng r;
    synth_rng_seed(&r, seed);
    sc->r0 = 0.9; sc->ru = 0.05; sc->rv = 0.03;
    const double lmin = log(8.0), lmax = log(512.0);
    int n = 0;
    for (int t = 0; t < n_tris; ++t) {
        synth_prim *q = &sc->p[n];
        for (;;) {
            const double x0 = rng_f64(&r), y0 = rng_f64(&r);
            const double l1 = exp(rng_range(&r, lmin, lmax)), a1 = rng_range(&r, 0.0, 2.0 * SYNTH_PI);
            const double l2 = exp(rng_range(&r, lmin, lmax)), a2 = rng_range(&r, 0.0, 2.0 * SYNTH_PI);
            const double x1 = x0 + l1 * cos(a1) / W, y1 = y0 + l1 * sin(a1) / H;
            const double x2 = x0 + l2 * cos(a2) / W, y2 = y0 + l2 * sin(a2) / H;
            if (x1 < 0.0 || x1 > 1.0 || y1 < 0.0 || y1 > 1.0) continue;
            if (x2 < 0.0 || x2 > 1.0 || y2 < 0.0 || y2 > 1.0) continue;
            q->kind = PRIM_POLY;
            q->nv = 3;
            q->x[0] = x0; q->y[0] = y0;
            q->x[1] = x1; q->y[1] = y1;
            q->x[2] = x2; q->y[2] = y2;
            break;
        }
        make_ccw(q);
        q->depth = rng_range(&r, 0.1, 0.8);
        ++n;
    }
    if (n_bars) {
        const double ang = rng_range(&r, 0.0, SYNTH_PI);
        const double nx = cos(ang), ny = sin(ang);
        const double depth = rng_range(&r, 0.1, 0.8);
        /* bar widths and gaps in texels, converted with the larger map side */
        const double texel = 1.0 / (double)(W > H ? W : H);
        double widths[64], gaps[64], extent = 0.0;
        for (int b = 0; b < n_bars; ++b) {
            widths[b] = rng_int(&r, 1, 3) * texel;
            gaps[b] = rng_int(&r, 8, 32) * texel;
            extent += widths[b] + gaps[b];
        }
        /* range of n.p over the unit square */
        double lo = 1e300, hi = -1e300;
        const double cxs[4] = {0, 1, 1, 0}, cys[4] = {0, 0, 1, 1};
        for (int k = 0; k < 4; ++k) {
            const double t = nx * cxs[k] + ny * cys[k];
            lo = t < lo ? t : lo;
            hi = t > hi ? t : hi;
        }
        const double slack = (hi - lo) - extent;
        double o = lo + (slack > 0.0 ? slack : 0.0) * rng_f64(&r);
        for (int b = 0; b < n_bars; ++b) {
            synth_prim *q = &sc->p[n++];
            q->kind = PRIM_SLAB;
            q->nx = nx; q->ny = ny;
            q->o = o; q->w = widths[b];
            q->depth = depth;
            o += widths[b] + gaps[b];
        }
    }
    sc->n = n;
    qsort(sc->p, (size_t)n, sizeof(synth_prim), cmp_depth);
    return sc;
}

/* Export the scene for other rasterizers: primitive k as the 112-byte record
 * {int32 kind, int32 nv, double x[4], y[4], nx, ny, o, w, float depth, int32 pad}
 * (kind 0: convex CCW polygon of nv vertices, 1: slab o <= nx*u + ny*v < o + w),
 * and the receiver plane (r0, ru, rv).  Returns the primitive count. */
typedef struct {
    int32_t kind, nv;
    double x[4], y[4];
    double nx, ny, o, w;
    float depth;
    int32_t pad;
} synth_prim_record;

int synth_scene_export(const synth_scene *sc, void *records, int cap, double receiver[3]) {
    synth_prim_record *out = (synth_prim_record *)records;
    for (int k = 0; k < sc->n && k < cap; ++k) {
        const synth_prim *q = &sc->p[k];
        synth_prim_record *r = &out[k];
        memset(r, 0, sizeof(*r));
        r->kind = q->kind;
        r->nv = q->nv;
        for (int e = 0; e < 4; ++e) { r->x[e] = q->x[e]; r->y[e] = q->y[e]; }
        r->nx = q->nx; r->ny = q->ny; r->o = q->o; r->w = q->w;
        r->depth = (float)q->depth;
    }
    if (receiver) { receiver[0] = sc->r0; receiver[1] = sc->ru; receiver[2] = sc->rv; }
    return sc->n;
}

/* Rasterize the scene into map[H][pitch] (float32).  Returns 0. */
int synth_scene_raster(const synth_scene *sc, float *map, int64_t pitch) {
    const int W = sc->W, H = sc->H;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i)
            map[(int64_t)j * pitch + i] = (float)receiver_depth(sc, (i + 0.5) / W, (j + 0.5) / H);
    for (int k = 0; k < sc->n; ++k) {
        const synth_prim *q = &sc->p[k];
        int i_lo = 0, i_hi = W - 1, j_lo = 0, j_hi = H - 1;
        if (q->kind == PRIM_POLY) {
            double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
            for (int e = 0; e < q->nv; ++e) {
                xmin = q->x[e] < xmin ? q->x[e] : xmin;
                xmax = q->x[e] > xmax ? q->x[e] : xmax;
                ymin = q->y[e] < ymin ? q->y[e] : ymin;
                ymax = q->y[e] > ymax ? q->y[e] : ymax;
            }
            i_lo = (int)floor(xmin * W) - 1; i_hi = (int)ceil(xmax * W) + 1;
            j_lo = (int)floor(ymin * H) - 1; j_hi = (int)ceil(ymax * H) + 1;
            i_lo = i_lo < 0 ? 0 : i_lo; j_lo = j_lo < 0 ? 0 : j_lo;
            i_hi = i_hi > W - 1 ? W - 1 : i_hi; j_hi = j_hi > H - 1 ? H - 1 : j_hi;
        }
        const float d = (float)q->depth;
        for (int j = j_lo; j <= j_hi; ++j) {
            const double py = (j + 0.5) / H;
            for (int i = i_lo; i <= i_hi; ++i) {
                const double px = (i + 0.5) / W;
                if (!prim_contains(q, px, py)) continue;
                float *t = &map[(int64_t)j * pitch + i];
                if (d < *t) *t = d;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fragments                                                                 */
/* ------------------------------------------------------------------------ */

/* n fragments with u, v i.i.d. uniform on [0,1) and constant depth z, packed
 * (u, v, z) as float32. */
void synth_frags_uniform(uint64_t seed, int64_t n, float z, float *out) {
    synth_rng r;
    synth_rng_seed(&r, seed);
    for (int64_t k = 0; k < n; ++k) {
        out[3 * k + 0] = rng_f32(&r);
        out[3 * k + 1] = rng_f32(&r);
        out[3 * k + 2] = z;
    }
}

typedef struct {
    double C[3];  /* camera position (u, v, z) in light space */
    double f[3], rt[3], up[3];
    double tx, ty;
} camera;

static void camera_ray(const camera *cam, int Ws, int Hs, double px, double py, double d[3]) {
    const double x = ((px + 0.5) / Ws) * 2.0 - 1.0;
    const double y = 1.0 - ((py + 0.5) / Hs) * 2.0;
    for (int k = 0; k < 3; ++k)
        d[k] = cam->f[k] + x * cam->tx * cam->rt[k] + y * cam->ty * cam->up[k];
}

/* Ray parameter where the ray meets the receiver plane. */
static double receiver_t(const synth_scene *sc, const camera *cam, const double d[3]) {
    const double *C = cam->C;
    const double num = sc->r0 + sc->ru * (C[0] - 0.5) + sc->rv * (C[1] - 0.5) - C[2];
    const double den = d[2] - sc->ru * d[0] - sc->rv * d[1];
    return num / den;
}

/* Project a light-space point to continuous pixel coordinates; returns 0 when
 * the point is not in front of the camera. */
static int project(const camera *cam, int Ws, int Hs, const double P[3], double *px, double *py) {
    double q[3];
    for (int k = 0; k < 3; ++k) q[k] = P[k] - cam->C[k];
    const double zc = q[0] * cam->f[0] + q[1] * cam->f[1] + q[2] * cam->f[2];
    if (zc <= 1e-9) return 0;
    const double xc = q[0] * cam->rt[0] + q[1] * cam->rt[1] + q[2] * cam->rt[2];
    const double yc = q[0] * cam->up[0] + q[1] * cam->up[1] + q[2] * cam->up[2];
    const double x = xc / (zc * cam->tx), y = yc / (zc * cam->ty);
    *px = (x + 1.0) * 0.5 * Ws - 0.5;
    *py = (1.0 - y) * 0.5 * Hs - 0.5;
    return 1;
}

/* Perspective camera over the scene, ray-cast in light space.  The camera looks
 * at the map centre with pitch 35 degrees from the light direction, vertical
 * field of view vfov_deg, square pixels, from depth 0.55; its yaw is a random
 * multiple of 90 degrees plus U(-8, 8) degrees.  Output: Ws*Hs fragments in
 * row-major screen order, (u, v, z) float32 of the first surface hit (the
 * nearest blocker, else the receiver).  Returns 0, or -1 when some pixel
 * lands outside [0,1)^2 (the placement guarantees it does not). */
static int camera_rows(const synth_scene *sc, uint64_t seed, int Ws, int Hs, double vfov_deg, int r0, int r1,
                       float *out);

int synth_frags_camera(const synth_scene *sc, uint64_t seed, int Ws, int Hs, double vfov_deg, float *out) {
    return camera_rows(sc, seed, Ws, Hs, vfov_deg, 0, Hs, out);
}

/* Rows [r0, r1) of the same camera image: (r1 - r0) * Ws fragments. */
int synth_frags_camera_rows(const synth_scene *sc, uint64_t seed, int Ws, int Hs, double vfov_deg, int r0, int r1,
                            float *out) {
    if (r0 < 0 || r1 > Hs || r0 > r1) return -3;
    return camera_rows(sc, seed, Ws, Hs, vfov_deg, r0, r1, out);
}

static int camera_rows(const synth_scene *sc, uint64_t seed, int Ws, int Hs, double vfov_deg, int r0, int r1,
                       float *out) {
    synth_rng r;
    synth_rng_seed(&r, seed);
    const double yaw = rng_int(&r, 0, 3) * (SYNTH_PI / 2.0) + rng_range(&r, -8.0, 8.0) * SYNTH_PI / 180.0;
    const double pitch = 35.0 * SYNTH_PI / 180.0;
    const double zc = 0.55;
    camera cam;
    const double h[3] = {cos(yaw), sin(yaw), 0.0};
    for (int k = 0; k < 3; ++k) {
        cam.f[k] = sin(pitch) * h[k] + (k == 2 ? cos(pitch) : 0.0);
        cam.up[k] = cos(pitch) * h[k] - (k == 2 ? sin(pitch) : 0.0);
    }
    cam.rt[0] = sin(yaw); cam.rt[1] = -cos(yaw); cam.rt[2] = 0.0;
    cam.ty = tan(0.5 * vfov_deg * SYNTH_PI / 180.0);
    cam.tx = cam.ty * (double)Ws / (double)Hs;
    const double target_z = receiver_depth(sc, 0.5, 0.5);
    const double s = (target_z - zc) / cam.f[2];
    cam.C[0] = 0.5 - s * cam.f[0];
    cam.C[1] = 0.5 - s * cam.f[1];
    cam.C[2] = zc;

    const int64_t npix = (int64_t)Ws * (r1 - r0);
    int32_t *winner = (int32_t *)malloc((size_t)(npix > 0 ? npix : 1) * sizeof(int32_t));
    if (!winner) return -2;
    for (int64_t k = 0; k < npix; ++k) winner[k] = -1;

    /* blockers in increasing depth: along a ray moving away from the light the
     * first one containing the ray's crossing point is the nearest hit */
    for (int k = 0; k < sc->n; ++k) {
        const synth_prim *q = &sc->p[k];
        if (q->depth <= zc) continue; /* behind the camera plane of motion */
        int x_lo = 0, x_hi = Ws - 1, y_lo = 0, y_hi = Hs - 1;
        if (q->kind == PRIM_POLY) {
            double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
            int ok = 1;
            for (int e = 0; e < q->nv && ok; ++e) {
                const double P[3] = {q->x[e], q->y[e], q->depth};
                double px = 0.0, py = 0.0;
                ok = project(&cam, Ws, Hs, P, &px, &py);
                if (!ok) break;
                xmin = px < xmin ? px : xmin; xmax = px > xmax ? px : xmax;
                ymin = py < ymin ? py : ymin; ymax = py > ymax ? py : ymax;
            }
            if (ok) {
                /* clamp before converting: a vertex near the camera plane projects far away */
                xmin = fmax(xmin, -2.0); xmax = fmin(xmax, (double)Ws + 1.0);
                ymin = fmax(ymin, -2.0); ymax = fmin(ymax, (double)Hs + 1.0);
                x_lo = (int)floor(xmin) - 1; x_hi = (int)ceil(xmax) + 1;
                y_lo = (int)floor(ymin) - 1; y_hi = (int)ceil(ymax) + 1;
                x_lo = x_lo < 0 ? 0 : x_lo; y_lo = y_lo < 0 ? 0 : y_lo;
                x_hi = x_hi > Ws - 1 ? Ws - 1 : x_hi; y_hi = y_hi > Hs - 1 ? Hs - 1 : y_hi;
            }
        }
        if (y_lo < r0) y_lo = r0;
        if (y_hi > r1 - 1) y_hi = r1 - 1;
        for (int py = y_lo; py <= y_hi; ++py) {
            for (int px = x_lo; px <= x_hi; ++px) {
                const int64_t idx = (int64_t)(py - r0) * Ws + px;
                if (winner[idx] >= 0) continue;
                double d[3];
                camera_ray(&cam, Ws, Hs, px, py, d);
                if (d[2] <= 0.0) continue;
                const double t = (q->depth - cam.C[2]) / d[2];
                if (t <= 0.0) continue;
                const double hu = cam.C[0] + t * d[0], hv = cam.C[1] + t * d[1];
                if (prim_contains(q, hu, hv)) winner[idx] = k;
            }
        }
    }

    int status = 0;
    for (int py = r0; py < r1; ++py) {
        for (int px = 0; px < Ws; ++px) {
            const int64_t idx = (int64_t)(py - r0) * Ws + px;
            double d[3];
            camera_ray(&cam, Ws, Hs, px, py, d);
            double u, v, z;
            if (winner[idx] >= 0) {
                const synth_prim *q = &sc->p[winner[idx]];
                const double t = (q->depth - cam.C[2]) / d[2];
                u = cam.C[0] + t * d[0];
                v = cam.C[1] + t * d[1];
                z = q->depth;
            } else {
                const double t = receiver_t(sc, &cam, d);
                u = cam.C[0] + t * d[0];
                v = cam.C[1] + t * d[1];
                z = receiver_depth(sc, u, v);
            }
            float fu = (float)u, fv = (float)v;
            if (!(fu >= 0.0f && fu < 1.0f && fv >= 0.0f && fv < 1.0f)) status = -1;
            out[3 * idx + 0] = fu;
            out[3 * idx + 1] = fv;
            out[3 * idx + 2] = (float)z;
        }
    }
    free(winner);
    return status;
}

int synth_scene_count(const synth_scene *sc) { return sc->n; }
