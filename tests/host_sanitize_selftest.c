/* Memory- and UB-sanitized run of the host C code: the seeded input
 * generator (synth/synth.c) and the oracle (oracle/rbsm_oracle.c), built
 * together with this driver by tests/test_host_sanitizers.py under
 * -fsanitize=address,undefined.  It exercises every oracle entry point the
 * tests use on small inputs, including fragments outside the map (clamped
 * reads), NaN texels and RPCF windows at the map's edge, and checks return
 * codes and output ranges; the sanitizers check every access. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct synth_scene synth_scene;
synth_scene *synth_scene_tris(uint64_t seed, int W, int H, int n_tris, int fence);
int synth_scene_raster(const synth_scene *sc, float *map, int64_t pitch);
int synth_scene_export(const synth_scene *sc, void *records, int cap, double receiver[3]);
int synth_frags_camera(const synth_scene *sc, uint64_t seed, int Ws, int Hs, double vfov_deg, float *out);
void synth_frags_uniform(uint64_t seed, int64_t n, float z, float *out);
void synth_scene_free(synth_scene *sc);

typedef struct {  /* the oracle's parameter record (same layout) */
    int32_t width, height;
    int64_t pitch;
    float depth_bias;
    int32_t max_dist;
    int32_t kernel_radius;
} oracle_params;
typedef struct {  /* the oracle's and the generator's primitive record (same layout) */
    int32_t kind, nv;
    double x[4], y[4];
    double nx, ny, o, w;
    float depth;
    int32_t pad;
} prim_record;
int oracle_shadow_map(const float *map, const float *frags, int64_t n, const oracle_params *p, uint8_t *out);
int oracle_rbsm_hard(const float *map, const float *frags, int64_t n, const oracle_params *p, uint8_t *out);
int oracle_rsmss(const float *map, const float *frags, int64_t n, const oracle_params *p, float *out);
double oracle_margin_one(const float *map, const float *frag, const oracle_params *p, int hard);
int oracle_raster(const prim_record *prims, int n, double r0, double ru, double rv, int W, int H, int64_t pitch,
                  float *map);
int oracle_composite(int64_t n, int n_lights, const void *const *vis, const int32_t *hard, const float *weights,
                     float *out);

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)

int main(void) {
    const int W = 96, H = 80, PITCH = 101, Ws = 40, Hs = 30;
    const int64_t n = (int64_t)Ws * Hs, nu = 500;
    synth_scene *sc = synth_scene_tris(7, W, H, 12, 1);
    CHECK(sc != NULL);
    float *map = malloc(sizeof(float) * (size_t)H * PITCH);
    for (int64_t k = 0; k < (int64_t)H * PITCH; ++k) map[k] = NAN;  /* padding past the width is never read */
    CHECK(synth_scene_raster(sc, map, PITCH) == 0);
    float *frags = malloc(sizeof(float) * 3 * (size_t)n);
    CHECK(synth_frags_camera(sc, 11, Ws, Hs, 50.0, frags) == 0);
    /* uniform fragments, some spilling past the map on every side */
    float *fu = malloc(sizeof(float) * 3 * (size_t)nu);
    synth_frags_uniform(13, nu, 0.5f, fu);
    for (int64_t k = 0; k < nu; k += 5) { fu[3 * k] = fu[3 * k] * 1.4f - 0.2f; fu[3 * k + 1] = fu[3 * k + 1] * 1.4f - 0.2f; }

    oracle_params p = {W, H, PITCH, 1e-3f, 16, 0};
    uint8_t *hard = malloc((size_t)n), *sm = malloc((size_t)n);
    float *soft = malloc(sizeof(float) * (size_t)n);
    CHECK(oracle_shadow_map(map, frags, n, &p, sm) == 0);
    CHECK(oracle_rbsm_hard(map, frags, n, &p, hard) == 0);
    CHECK(oracle_rsmss(map, frags, n, &p, soft) == 0);
    for (int64_t k = 0; k < n; ++k) CHECK(hard[k] <= 1 && soft[k] >= 0.0f && soft[k] <= 1.0f);
    for (int64_t k = 0; k < n; k += 37) CHECK(oracle_margin_one(map, frags + 3 * k, &p, k & 1) >= 0.0);

    uint8_t *hu = malloc((size_t)nu);
    float *su = malloc(sizeof(float) * (size_t)nu);
    oracle_params pm = {W, H, PITCH, 0.0f, 64, 0};
    CHECK(oracle_rbsm_hard(map, fu, nu, &pm, hu) == 0);
    CHECK(oracle_rsmss(map, fu, nu, &pm, su) == 0);

    /* RPCF windows at and past the map's edges */
    oracle_params pr = {W, H, PITCH, 1e-3f, 8, 5};
    float *rp = malloc(sizeof(float) * (size_t)nu);
    CHECK(oracle_rsmss(map, fu, 200, &pr, rp) == 0);
    for (int64_t k = 0; k < 200; ++k) CHECK(rp[k] >= 0.0f && rp[k] <= 1.0f);

    /* NaN texels (lit at every depth) inside the map */
    for (int j = 10; j < 20; ++j) map[(int64_t)j * PITCH + 30] = NAN;
    CHECK(oracle_rbsm_hard(map, frags, n, &p, hard) == 0);
    CHECK(oracle_rsmss(map, frags, n, &p, soft) == 0);

    /* rasterization from the exported primitives, and compositing */
    prim_record recs[64];
    double rec[3];
    const int np = synth_scene_export(sc, recs, 64, rec);
    CHECK(np > 0 && np <= 64);
    float *map2 = malloc(sizeof(float) * (size_t)H * W);
    CHECK(oracle_raster(recs, np, rec[0], rec[1], rec[2], W, H, W, map2) == 0);
    const void *vis[2] = {hard, soft};
    const int32_t modes[2] = {1, 0};
    const float wts[2] = {0.25f, 0.75f};
    float *comp = malloc(sizeof(float) * (size_t)n);
    CHECK(oracle_composite(n, 2, vis, modes, wts, comp) == 0);

    free(comp); free(map2); free(rp); free(su); free(hu); free(soft); free(sm); free(hard); free(fu); free(frags);
    free(map);
    synth_scene_free(sc);
    printf("host sanitize ok\n");
    return 0;
}
