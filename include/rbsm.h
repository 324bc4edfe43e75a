/*
 * rbsm.h -- C ABI of the MI355X (gfx950) revectorization-based shadow mapping
 * pass: hard silhouette recovery (SMSR) and revectorization-based filtering
 * (RSMSS) from Macedo, Apolinario, Aguero, "Optimized Visibility Functions for
 * Revectorization-Based Shadow Mapping" (arXiv 1711.07793).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is DEVICE memory owned by the caller.  The
 * library keeps no pointer after the enqueued work completes and allocates no
 * device memory per call.  Outputs must not overlap any input; overlapping
 * ranges are rejected.
 *
 * Streams.  Work is enqueued on `stream` (0 = the default stream) and runs
 * asynchronously; completion is observed with stream or event synchronisation.
 * Argument checks happen on the host before anything is enqueued.
 *
 * Shadow map.  float32, row-major, texel (i, j) at shadow_map[j*pitch + i],
 * 0 <= i < width, 0 <= j < height; row j holds v-texel j and +j is "top"
 * (the +y neighbour of the discontinuity listing, Sec. 3.1.2).
 *
 * Fragments.  n camera fragments already in light space (the varying p of
 * Listing 1, Sec. 3), packed as float32 (u, v, z) triples: u, v texture
 * coordinates, z the fragment's light-space depth.  Inputs must be finite.
 * Addressing is nearest-texel: X = u*width (binary32), texel floor(X),
 * sub-texel fraction X - floor(X); every texel read is clamped to the map
 * (clamp-to-edge), so u, v outside [0, 1) are legal.
 *
 * Shadow test (Eq. 1).  A texel of depth T is lit for a fragment of depth z
 * unless (z - depth_bias) > T, z - depth_bias rounded to binary32 once.
 *
 * Errors.  Entry points return RBSM_OK (0) or a negative code; nothing is
 * enqueued on error.  rbsm_last_error() returns a thread-local message for
 * the calling thread's last failure.  No C++ exception crosses this ABI.
 * Entry points are reentrant and thread-safe.
 */
#ifndef RBSM_H
#define RBSM_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RBSM_OK = 0,
    RBSM_ERR_INVALID_ARG = -1, /* bad pointer, size, parameter or overlap */
    RBSM_ERR_HIP = -2          /* the HIP runtime reported an error */
};

/* Parameters of one pass (read at call time). */
typedef struct {
    int32_t width, height;  /* shadow map size in texels, 1..65536 each */
    int64_t pitch;          /* floats between consecutive map rows, >= width */
    float depth_bias;       /* subtracted from z before the test; 0 = Eq. 1 exactly */
    int32_t max_dist;       /* MAXDIST of the traversal listing (Sec. 3.1.3), 1..64 */
    int32_t kernel_radius;  /* RSMSS only: 0 = Listing 5 exactly, r > 0 = RPCF box
                               average over (2r+1)^2 texel offsets, 0..32 */
    int32_t view_width;     /* layout hint, never changes a result: > 0 when the
                               fragments are a row-major image of this many
                               columns (fragment k is pixel (k % view_width,
                               k / view_width); the last row may be partial), so
                               the pass can work in 2-D screen tiles whose
                               light-space footprint is staged in LDS; 0 = no
                               layout (flat chunks) */
} rbsm_params;

/*
 * Hard RBSM: shadow silhouette recovery (Sec. 3.1; Listings 1-4).
 * Shadowed fragments stay shadowed; a lit fragment on a shadow edge is
 * classified by the bounded edge traversal and the normalized discontinuity
 * space, then put in shadow by the shape rules of Listing 4 (U/O shadowed,
 * I lit, L clipped by the revectorization line nrd.y < 1 - nrd.x).
 *   shadow_map  [height*pitch] float32, read only
 *   frags       [3*n] float32 (u, v, z), read only
 *   n           number of fragments, >= 0 (0 is a no-op)
 *   p           parameters; p->kernel_radius must be 0
 *   out_mask    [n] uint8 written: 0 = shadow, 1 = lit, in fragment order
 */
int rbsm_visibility(const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                    uint8_t *out_mask, hipStream_t stream);

/*
 * RSMSS: revectorization-based shadow filtering (Sec. 3.2; Listings 1-3, 5).
 * Every fragment is classified (lit and shadowed sides); the result is the
 * fixed-size fake penumbra in [0, 1].  With p->kernel_radius = r > 0 the
 * result is the RPCF box average: the RSMSS value evaluated at each of the
 * (2r+1)^2 texels (i0+a, j0+b), |a|, |b| <= r, with the fragment's own
 * sub-texel position and depth, averaged (PCF over the filtered edge,
 * Sec. 5.3): the exact mean of those binary32 values rounded to binary32.
 * It is computed as a binary64 sum in an unspecified order divided once by
 * (2r+1)^2, which stays within 5e-13 of the exact mean, so the result is the
 * rounded exact mean except at a near-tie, where it may be the neighbouring
 * binary32 value.
 *   out_vis     [n] float32 written: visibility in [0, 1], fragment order
 * Other arguments as rbsm_visibility.
 */
int rsmss_visibility(const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                     float *out_vis, hipStream_t stream);

/*
 * Plain shadow mapping (Eq. 1 at the fragment's texel; Williams 1978), the
 * baseline the paper compares RBSM against (Tables 2-5).
 *   out_mask    [n] uint8 written: 0 = shadow, 1 = lit
 * p->max_dist and p->kernel_radius are ignored.
 */
int sm_visibility(const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                  uint8_t *out_mask, hipStream_t stream);

/*
 * Read-set instrumentation (no visibility output): marks with 1 every texel
 * the pass reads for these fragments, as the paper's listings read them --
 * the fragment's texel; unless hard mode stops at a shadowed texel, its four
 * neighbours; for each traversal step, the visited texel and, when it has the
 * fragment's test result, that texel's four neighbours.  Used to count the
 * distinct texels a pass touches (its algorithmic map bytes).
 *   mode        0 = hard (rbsm_visibility), 1 = RSMSS (rsmss_visibility)
 *   touched     [height*width] uint8, row-major without pitch; the caller
 *               clears it; entries are only ever set to 1
 */
int rbsm_footprint(const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                   int32_t mode, uint8_t *touched, hipStream_t stream);

/*
 * Launch tuning of the hard / RSMSS (radius 0) pass.  Tuning never changes a
 * result, only which lanes read which texels from where; it is what the
 * project's autotuner searches.
 */
typedef struct {
    int32_t tile_w;     /* screen-tile width in pixels: 16, 32 or 64 (height 1024 / tile_w);
                           ignored (flat 1024-fragment chunks) when view_width is 0 */
    int32_t apron;      /* texels staged around the tile's texel box, 1..8 */
    int32_t lds_cap;    /* LDS texel capacity per workgroup, 256..12288, or 0:
                           nothing staged, every texel read from global memory */
    int32_t persistent; /* 0: one workgroup per screen tile; 1: only resident
                           workgroups, looping over tiles: in plans of up to 48
                           jobs with tiles they take tiles from one queue per XCD;
                           otherwise (and in the plain entry points) each takes a
                           fixed share and loads the next tile's fragments while
                           it works on the current one */
    int32_t walk_first; /* traversal steps every walk takes before unfinished
                           walks are regrouped: 1, 2 or 4 (0 = default 2) */
    int32_t walk_block; /* steps per block of a regrouped walk, read together:
                           4 or 8 (0 = default 4); with persistent = 1 both
                           walk fields must be 0 or their defaults */
    int32_t xcd_chunk;  /* how tiles are dealt to the 8 XCDs: -1 one contiguous
                           range each; c in 0..12: chunks of 2^c consecutive
                           tiles round-robin (balances uneven jobs) */
} rbsm_tuning;

/* The tuning the plain entry points use. */
rbsm_tuning rbsm_default_tuning(void);

/*
 * rbsm_visibility (mode 0, out = uint8_t[n]) or rsmss_visibility with
 * kernel_radius 0 (mode 1, out = float[n]) under an explicit tuning.
 * Arguments as those entry points; tune must be valid (RBSM_ERR_INVALID_ARG
 * otherwise).  This entry point honours tile_w, apron, lds_cap and
 * persistent; walk_first and walk_block must be 0 or their defaults (the
 * walk blocking is searched in plans, whose kernels are built for each).
 */
int rbsm_pass_tuned(int32_t mode, const float *shadow_map, const float *frags, int64_t n,
                    const rbsm_params *p, const rbsm_tuning *tune, void *out, hipStream_t stream);

/*
 * Batched form: many (view, light) passes of uneven sizes in one launch.
 * Every job is a hard (mode 0) or RSMSS (mode 1) pass over its own map,
 * fragments and output.  The hard and RSMSS radius-0 jobs share one launch of
 * the tile pass over every screen tile of every job (one workgroup per tile,
 * or resident workgroups looping over them), so small jobs share the GPU with
 * large ones; RSMSS jobs with kernel_radius > 0 (RPCF, Sec. 5.3) run the
 * box-filter kernel, one launch each, before it.  A frame is one call (or one
 * graph replay).  Each output is bitwise the result of the corresponding
 * plain entry point.
 */
typedef struct {
    const float *shadow_map;  /* device, as rbsm_visibility */
    const float *frags;       /* device, [3*n] */
    int64_t n;                /* fragments, >= 0 */
    rbsm_params params;       /* kernel_radius 0, or > 0 for an RPCF job (mode 1) */
    int32_t mode;             /* 0: hard, out is uint8_t[n]; 1: RSMSS, out is float[n] */
    void *out;                /* device; must not overlap any input or other output */
} rbsm_job;

typedef struct rbsm_plan rbsm_plan;  /* opaque; owns device tables */

/* Build a plan for n_jobs (1..65535) jobs; tune may be NULL (defaults).
 * Copies the job table to the device (synchronous).  On success *plan owns
 * device memory until rbsm_plan_destroy. */
int rbsm_plan_create(const rbsm_job *jobs, int32_t n_jobs, const rbsm_tuning *tune, rbsm_plan **plan);

/* Replace the jobs (pointers, depth, bias...) keeping each job's fragment
 * count, view_width and kernel_radius, so the tile layout is unchanged
 * (synchronous copy; call when no launch of the plan is in flight).  A
 * captured graph is captured again with the new jobs (on a stream the call
 * creates and destroys), so later replays use them. */
int rbsm_plan_update(rbsm_plan *plan, const rbsm_job *jobs, int32_t n_jobs);

/* Enqueue one batched pass on stream (graph replay after rbsm_plan_capture). */
int rbsm_plan_launch(rbsm_plan *plan, hipStream_t stream);

/* Project autotuner.  Times candidate tunings over reps launches each on
 * stream with HIP events and keeps the fastest, searching one axis after the
 * other: tile width x launch form (one workgroup per tile or persistent),
 * then (one workgroup per tile) the XCD chunking, then LDS capacity, then
 * apron, then (one workgroup per tile) the walk blocking; a candidate
 * replaces the best only when it is more than 2% faster, so near-ties keep
 * the earlier choice in this order.  The
 * choice is cached in the process under a key of the device (architecture,
 * CU count) and the plan's job layout (per job: fragments, view width, map
 * size and pitch, MAXDIST, mode); a later call with the same key applies the
 * cached tuning without timing unless flags bit 0 (RBSM_TUNE_FORCE) is set.
 * Writes the tuning to *chosen when non-NULL.  Outputs are recomputed, never
 * changed.  Drops a captured graph. */
enum { RBSM_TUNE_FORCE = 1 };
int rbsm_plan_autotune(rbsm_plan *plan, hipStream_t stream, int32_t reps, int32_t flags, rbsm_tuning *chosen);

/* The autotuner cache as a text file (one line per key: key tile_w apron
 * lds_cap persistent walk_first walk_block xcd_chunk).  load returns the number of
 * entries read (>= 0) or a negative code (unreadable file, malformed or
 * invalid entry: entries before it stay loaded); save writes every entry. */
int rbsm_tune_cache_load(const char *path);
int rbsm_tune_cache_save(const char *path);
void rbsm_tune_cache_clear(void);

int rbsm_plan_set_tuning(rbsm_plan *plan, const rbsm_tuning *tune);  /* drops a captured graph */
int rbsm_plan_get_tuning(const rbsm_plan *plan, rbsm_tuning *tune);

/* Capture the plan's launch on stream (not the default stream) into a HIP
 * graph; later rbsm_plan_launch calls on any stream replay it. */
int rbsm_plan_capture(rbsm_plan *plan, hipStream_t stream);

/* Total fragments over the plan's jobs (-1 for a null plan). */
int64_t rbsm_plan_fragments(const rbsm_plan *plan);

void rbsm_plan_destroy(rbsm_plan *plan);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one batched
 * pass of `jobs`, as rbsm_plan_create + rbsm_plan_launch + rbsm_plan_destroy
 * would run it (bitwise the same outputs), that allocates nothing.  The job
 * table and the tile -> job map live in a 4 MiB array of the library's own
 * in device memory, one per GPU, held until the process ends, and are
 * rewritten by every call (job records travel in kernel arguments).
 *   jobs, n_jobs   as rbsm_plan_create, at most 4096 jobs and 1,916,928
 *                  screen tiles (about 1.9e9 fragments); larger requests
 *                  return RBSM_ERR_INVALID_ARG before anything is enqueued
 *   tune           NULL (defaults) or a valid tuning
 *   stream         as the other entry points (asynchronous)
 * Calls on one GPU share its array: a call's kernels must not overlap
 * another call's on the same GPU (serialise them on one stream, or wait).
 */
int rbsm_batch_launch_noalloc(const rbsm_job *jobs, int32_t n_jobs, const rbsm_tuning *tune, hipStream_t stream);

/*
 * Shadow-map rasterization on the device: the light pass that produces the
 * depth map the pass consumes (Sec. 2 takes it as given), so a frame can stay
 * on the GPU from scene to visibility.
 *
 * Texel (i, j) samples its centre u = (i + 0.5) / width, v = (j + 0.5) /
 * height and stores the nearest surface there: the minimum of the receiver
 * plane r0 + ru (u - 0.5) + rv (v - 0.5) (evaluated in binary64, rounded to
 * binary32) and the depth of every primitive covering the centre; among equal
 * depths (+0 and -0 compare equal; a NaN depth never wins) the plane, then the
 * primitive of lowest index, is kept.  A convex
 * polygon (vertices counter-clockwise in (u, v)) covers a point when no edge
 * function (b - a) x (p - a) is negative and each zero lies on an edge that
 * runs downwards or horizontally to the left (top-left tie rule); a slab
 * covers o <= nx u + ny v < o + w.  Coverage is decided in binary64 without
 * contraction.  Primitives of another kind or vertex count cover nothing.
 */
typedef struct {
    int32_t kind;        /* 0: convex polygon, 1: slab */
    int32_t nv;          /* polygon vertex count, 3 or 4 */
    double x[4], y[4];   /* polygon vertices in texture coordinates */
    double nx, ny, o, w; /* slab: unit normal and the covered range of n.p */
    float depth;         /* constant light-space depth */
    int32_t pad;         /* unused */
} rbsm_prim;             /* 112 bytes */

/*
 *   prims       [n_prims] device array of rbsm_prim, read only
 *   n_prims     >= 0
 *   r0, ru, rv  receiver plane
 *   shadow_map  [height*pitch] float32 device output, row-major (columns >=
 *               width untouched); must not overlap prims.  Any alignment is
 *               accepted; a 16-byte-aligned map with pitch a multiple of 4
 *               is written with 16-byte stores (faster)
 */
int rbsm_rasterize(const rbsm_prim *prims, int32_t n_prims, double r0, double ru, double rv, int32_t width,
                   int32_t height, int64_t pitch, float *shadow_map, hipStream_t stream);

/*
 * Multi-light compositing: one shadow value per fragment of a view lit by
 * several lights, the weighted sum of the per-light visibilities,
 *   out[k] = sum over l in order of weights[l] * vis_l[k]
 * in binary32 (each product rounded, then added).  The visibility function
 * scales one light's contribution (Listing 1); how several lights combine is
 * not in the paper, so the weights are the caller's per-light intensities.
 *   n          fragments, >= 0 (0 is a no-op)
 *   n_lights   1..8
 *   vis        host array of n_lights DEVICE pointers: uint8_t[n] masks from
 *              rbsm_visibility (modes[l] = 0) or float[n] from
 *              rsmss_visibility (modes[l] = 1)
 *   modes, weights  host arrays of n_lights
 *   out        device float[n]; must not overlap any vis array
 * Any alignment is accepted; with masks 4-byte aligned and float arrays and
 * out 16-byte aligned, 4 fragments move per load and store (faster), with
 * the same results.
 */
int rbsm_composite(int64_t n, int32_t n_lights, const void *const *vis, const int32_t *modes, const float *weights,
                   float *out, hipStream_t stream);

/*
 * Serving engine: continuous batching of shadow requests over resident maps.
 *
 * An engine owns one device arena of hbm_budget_bytes, allocated at creation
 * (the only device allocation it makes), three streams (compute, upload,
 * copy-back) and a scheduler thread.  A request is one view: its light-space
 * fragments for 1..8 registered lights, plus buffers for the results.
 * Fragments in device memory of the engine's device are read in place;
 * fragments in host memory (pinned memory overlaps best) are uploaded into
 * the arena on the upload stream while earlier steps compute.  A result
 * buffer in device memory is written in place; a host buffer is staged in the
 * arena and copied back on the copy stream while the next step computes.
 *
 * Admission (first come, first served): a request is admitted while fewer
 * than max_inflight are, its staged buffers fit in the arena, and the HBM
 * working sets of all admitted requests -- every light's fragments (12 B per
 * fragment) and result (1 or 4 B), and the composite (4 B), wherever they
 * live -- stay within hbm_budget_bytes.  Each scheduling step runs one
 * batched pass over the jobs of every admitted request (each per-light result
 * is bitwise the plain entry point's), the RPCF jobs, and one compositing
 * launch.  Requests that arrive while others run join the next step.
 * Results are the same alone and in any mix.
 *
 * Stream order: a request's kernels wait for everything enqueued on its
 * `stream` before the submit call (an event recorded there), so fragments
 * and result buffers may be produced or last used asynchronously on it.
 */
typedef struct rbsm_engine rbsm_engine;  /* opaque */

typedef struct {
    int32_t light;         /* id from rbsm_engine_add_light */
    int32_t mode;          /* 0: hard (rbsm_visibility), 1: RSMSS / RPCF (rsmss_visibility) */
    const float *frags;    /* [3*n] light-space (u, v, z) for this light: device memory
                              (read in place) or host memory (uploaded) */
    float depth_bias;
    int32_t max_dist;      /* 1..64 */
    int32_t kernel_radius; /* mode 1 only, 0..32 */
    float weight;          /* this light's weight in the composite */
    void *out;             /* uint8_t[n] (mode 0) or float[n] (mode 1) for this light's
                              result, or NULL; device memory (written in place, must
                              not overlap any input) or host memory (pinned overlaps
                              best) */
} rbsm_request_light;

typedef struct {
    int64_t n;             /* fragments of the view, 0..2^31-1 */
    int32_t view_width;    /* layout hint as in rbsm_params */
    int32_t n_lights;      /* 1..8 */
    rbsm_request_light lights[8];
    float *composite;      /* float[n] for the composite, or NULL; device or host as `out` */
    hipStream_t stream;    /* the caller's stream that produced the device inputs and last
                              used the device result buffers (0 = the default stream) */
} rbsm_request;

typedef struct {
    int64_t submitted, completed, queued, inflight;
    int64_t launches, jobs_launched;  /* scheduling steps, (request, light) jobs */
    int64_t fragments_completed;      /* sum over completed requests of n * n_lights */
    int64_t arena_bytes, arena_peak_bytes;
    int64_t gpu_busy_ns;              /* summed GPU time of the scheduling steps' compute */
    int64_t inflight_bytes;           /* HBM working set of the admitted requests now */
    int64_t inflight_peak_bytes;      /* its largest value so far (<= the budget) */
    int64_t uploaded_bytes;           /* host fragments uploaded into the arena */
} rbsm_engine_stats;

/* Create an engine on the current device.  hbm_budget_bytes >= 4096,
 * max_inflight 1..4096. */
int rbsm_engine_create(int64_t hbm_budget_bytes, int32_t max_inflight, rbsm_engine **engine);

/* Register a resident shadow map (device, caller-owned, row-major with pitch;
 * must stay valid while the engine uses it).  Writes its id. */
int rbsm_engine_add_light(rbsm_engine *engine, const float *shadow_map, int32_t width, int32_t height, int64_t pitch,
                          int32_t *light_id);

/* Queue a request (copied; the arrays it points to are not).  Rejected when
 * its working set alone exceeds the budget, or a device result buffer
 * overlaps an input.  Writes a ticket. */
int rbsm_engine_submit(rbsm_engine *engine, const rbsm_request *request, int64_t *ticket);

/* Wait up to timeout_ms (< 0: forever) for a ticket.  Returns 1 when all its
 * results are in their buffers (the ticket is then forgotten and
 * *latency_ms, if non-NULL, is submit-to-completion time), 0 on time-out, a
 * negative code on failure. */
int rbsm_engine_wait(rbsm_engine *engine, int64_t ticket, int32_t timeout_ms, double *latency_ms);

int rbsm_engine_get_stats(rbsm_engine *engine, rbsm_engine_stats *stats);

/* Stop serving: every queued and admitted request completes with an error
 * (rbsm_engine_wait returns a negative code) once the work already enqueued
 * for it has finished, so no buffer is written after its wait returns; later
 * submissions are rejected.  For callers that must abort, and for tests of
 * the failure path. */
int rbsm_engine_abort(rbsm_engine *engine, const char *reason);

/* Finish every queued request, stop the scheduler and free the engine. */
void rbsm_engine_destroy(rbsm_engine *engine);

/* Message for the calling thread's last non-zero return ("" if none). */
const char *rbsm_last_error(void);

/* ABI version: 100 * major + minor (1.02: compositing, the serving engine and
 * rasterization; 1.03: persistent launches, walk blocking, XCD chunking, the
 * tuning cache, RPCF jobs in plans, the allocation-free batched pass, host
 * fragments and producer streams in the engine, engine abort). */
int32_t rbsm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RBSM_H */
