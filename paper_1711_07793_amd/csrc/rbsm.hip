// RBSM / RSMSS per-fragment shadow pass for MI355X (gfx950) and its C ABI.
//
// The main hard / RSMSS pass lives in tile_pass.hpp, the RPCF box filter in
// rpcf_pass.hpp; this file holds the plain shadow-map and read-set kernels,
// argument validation, the batched plan and the exported entry points (their
// contract is in rbsm.h).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rbsm.h"
#include "rbsm_device.hpp"
#include "tile_pass.hpp"
#include "rpcf_pass.hpp"
#include "raster_pass.hpp"

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
    int64_t grid = 0;  // workgroups of a persistent launch (resident ones, at most blocks)
    std::vector<int32_t> rpcf_jobs;  // jobs with kernel_radius > 0, launched before the tile pass
    BatchArgs args{};                // the tile-pass jobs as kernel arguments (when use_args)
    bool use_args = false;
    int *d_counters = nullptr;       // per-XCD tile queues of a persistent launch (zero between launches)
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
    if (p->d_counters) (void)hipFree(p->d_counters);
    p->d_jobs = nullptr;
    p->d_block_job = nullptr;
    p->d_counters = nullptr;
}

int64_t plan_grid(const rbsm_plan *p);

// Validate jobs and build (and upload) the device job table and the
// block -> job map for the plan's tile width.
// Host-side tables of a batch: the device job records, the block -> job map
// of the tile pass (when wanted) and the RPCF jobs, after validating every
// job and every overlap.
struct HostTables {
    std::vector<JobDev> dev;
    std::vector<int64_t> job_tiles;  // tiles of each job in the tile pass (0 for RPCF and empty jobs)
    std::vector<uint16_t> block_job;
    std::vector<int32_t> rpcf;
    std::vector<int32_t> order;      // the jobs in the order of their tiles
    int64_t tiles = 0, frags = 0;
    int tile_w = 32;
};

// The jobs with tiles as kernel-argument records, when there are at most
// kArgJobsMax of them, every pitch fits 32 bits and every job fits the 32-bit
// index form of the pass.
bool make_args(const HostTables &T, BatchArgs *a) {
    int k = 0;
    for (const int32_t j : T.order) {
        if (T.job_tiles[j] == 0) continue;
        const JobDev &D = T.dev[j];
        if (k == kArgJobsMax || D.m.pitch > (int64_t)INT32_MAX || !index32(D.n, D.vw, T.tile_w)) return false;
        JobArg &A = a->jobs[k];
        A.t = D.m.t;
        A.frags = D.frags;
        A.out = D.out;
        A.pitch = (int32_t)D.m.pitch;
        A.W = D.m.W;
        A.H = D.m.H;
        A.n = (int32_t)D.n;
        A.vw = (int32_t)D.vw;
        A.tiles_x = (int32_t)D.tiles_x;
        A.tile_base = (int32_t)D.tile_base;
        A.bias = D.bias;
        A.maxd = (int16_t)D.maxd;
        A.vec_ok = (uint8_t)D.vec_ok;
        A.mode = (uint8_t)D.mode;
        a->first[k] = (int32_t)D.tile_base;
        ++k;
    }
    for (int r = k; r < kArgJobsMax; ++r) a->first[r] = INT32_MAX;
    return k > 0;
}

// With rsmss_first, the tiles of RSMSS jobs come before those of hard jobs
// (each kind in job order): the launch then ends on the lighter hard tiles,
// which shortens its tail (a batched frame of cascades and spot lights
// measured 2-3% faster).  Otherwise tiles follow job order, as the
// allocation-free path's per-tile search over the job table needs.
int make_tables(const char *fn, const rbsm_job *jobs, int32_t n_jobs, int tile_w, const std::vector<rbsm_job> *same_layout,
                bool want_map, bool rsmss_first, HostTables &T) {
    if (!jobs || n_jobs < 1 || n_jobs > 65535) return fail(RBSM_ERR_INVALID_ARG, "%s: need 1..65535 jobs", fn);
    if (same_layout && (size_t)n_jobs != same_layout->size())
        return fail(RBSM_ERR_INVALID_ARG, "%s: job count differs from the plan", fn);
    T.dev.assign(n_jobs, JobDev{});
    T.job_tiles.assign(n_jobs, 0);
    T.tile_w = tile_w;
    T.block_job.clear();
    T.rpcf.clear();
    T.order.clear();
    int64_t frags = 0;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const rbsm_job &J = jobs[j];
        if (J.mode != 0 && J.mode != 1) return fail(RBSM_ERR_INVALID_ARG, "%s: job mode must be 0 or 1", fn);
        MapView mv;
        const int st = validate(fn, J.shadow_map, J.frags, J.n, &J.params, J.out, J.mode == 0 ? 1 : 4, J.mode == 1,
                                &mv);
        if (st != RBSM_OK) return st;
        if (same_layout && (J.n != (*same_layout)[j].n || J.params.view_width != (*same_layout)[j].params.view_width ||
                            J.params.kernel_radius != (*same_layout)[j].params.kernel_radius))
            return fail(RBSM_ERR_INVALID_ARG, "%s: a job's n, view_width or kernel_radius differs from the plan", fn);
        // RPCF jobs (radius > 0) run their own kernel: no tiles in the tile pass
        const bool rpcf = J.mode == 1 && J.params.kernel_radius > 0;
        JobLayout L = job_layout(J.n, J.params.view_width, tile_w);
        if (rpcf) {
            L.tiles = 0;
            T.rpcf.push_back(j);
        }
        JobDev &D = T.dev[j];
        D.m = mv;
        D.frags = J.frags;
        D.out = J.out;
        D.n = J.n;
        D.vw = L.vw;
        D.tiles_x = L.tiles_x;
        D.bias = J.params.depth_bias;
        D.maxd = J.params.max_dist;
        D.mode = J.mode;
        D.vec_ok = ((uintptr_t)J.frags % 16 == 0) && ((uintptr_t)J.out % (J.mode == 0 ? 4 : 16) == 0) &&
                   (L.vw % 4 == 0);
        T.job_tiles[j] = L.tiles;
        frags += J.n;
    }
    for (int pass = rsmss_first ? 0 : 1; pass < 2; ++pass)
        for (int32_t j = 0; j < n_jobs; ++j)
            if (!rsmss_first || (jobs[j].mode == 1) == (pass == 0)) T.order.push_back(j);
    int64_t base = 0;
    for (const int32_t j : T.order) {
        T.dev[j].tile_base = base;
        if (want_map)
            for (int64_t b = 0; b < T.job_tiles[j]; ++b) T.block_job.push_back((uint16_t)j);
        base += T.job_tiles[j];
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
    T.tiles = base;
    T.frags = frags;
    return RBSM_OK;
}

int build_tables(rbsm_plan *plan, const rbsm_job *jobs, int32_t n_jobs, bool keep_layout) {
    const char *fn = keep_layout ? "rbsm_plan_update" : "rbsm_plan_create";
    HostTables T;
    const int st = make_tables(fn, jobs, n_jobs, plan->tune.tile_w, keep_layout ? &plan->jobs : nullptr, true, true, T);
    if (st != RBSM_OK) return st;
    const int64_t base = T.tiles;
    if (!keep_layout || base != plan->blocks) {
        free_tables(plan);
        constexpr size_t kCounterBytes = 8 * 16 * sizeof(int);  // one queue counter per XCD, 64 bytes apart
        if (hipMalloc(&plan->d_jobs, sizeof(JobDev) * (size_t)n_jobs) != hipSuccess ||
            hipMalloc(&plan->d_block_job, sizeof(uint16_t) * (size_t)std::max<int64_t>(base, 1)) != hipSuccess ||
            hipMalloc(&plan->d_counters, kCounterBytes) != hipSuccess ||
            hipMemset(plan->d_counters, 0, kCounterBytes) != hipSuccess) {
            free_tables(plan);
            return fail(RBSM_ERR_HIP, "%s: could not allocate the job tables", fn);
        }
    }
    if (hipMemcpy(plan->d_jobs, T.dev.data(), sizeof(JobDev) * (size_t)n_jobs, hipMemcpyHostToDevice) != hipSuccess ||
        (base > 0 && hipMemcpy(plan->d_block_job, T.block_job.data(), sizeof(uint16_t) * (size_t)base,
                               hipMemcpyHostToDevice) != hipSuccess))
        return fail(RBSM_ERR_HIP, "%s: could not upload the job tables", fn);
    plan->jobs.assign(jobs, jobs + n_jobs);
    plan->rpcf_jobs = T.rpcf;
    plan->use_args = make_args(T, &plan->args);
    plan->blocks = base;
    plan->fragments = T.frags;
    plan->grid = plan_grid(plan);
    return RBSM_OK;
}

// Batched kernel instances: one workgroup per tile with the job records in a
// device table (batch_kernel) or in the kernel arguments (batch_arg_kernel),
// each built for every walk blocking the tuner tries, or resident workgroups
// looping over the tiles (batch_persistent_kernel).
template <int TW, int WF, int WB>
struct TableKernel {
    static const void *get() { return reinterpret_cast<const void *>(&batch_kernel<TW, WF, WB>); }
};
template <int TW, int WF, int WB>
struct ArgKernel {
    static const void *get() { return reinterpret_cast<const void *>(&batch_arg_kernel<TW, WF, WB>); }
};

// Kernel K<TW, WF, WB> for a tuning's walk blocking.
template <template <int, int, int> class K, int TW>
const void *walk_instance(int wf, int wb) {
    if (wb == 8) {
        if (wf == 1) return K<TW, 1, 8>::get();
        if (wf == 4) return K<TW, 4, 8>::get();
        return K<TW, 2, 8>::get();
    }
    if (wf == 1) return K<TW, 1, 4>::get();
    if (wf == 4) return K<TW, 4, 4>::get();
    return K<TW, 2, 4>::get();
}

template <template <int, int, int> class K>
const void *width_instance(int tw, int wf, int wb) {
    if (tw == 16) return walk_instance<K, 16>(wf, wb);
    if (tw == 64) return walk_instance<K, 64>(wf, wb);
    return walk_instance<K, 32>(wf, wb);
}

// The kernel a tuning launches, with the job records in the kernel arguments
// (args) or in device tables: persistent launches use the default walk
// blocking (one instance per tile width).
const void *batch_instance(const rbsm_tuning &t, bool args) {
    const int wf = t.walk_first ? t.walk_first : kWalkFirst, wb = t.walk_block ? t.walk_block : kWalkSteps;
    if (t.persistent && args) {
        if (t.tile_w == 16) return reinterpret_cast<const void *>(&batch_arg_queue_kernel<16>);
        if (t.tile_w == 64) return reinterpret_cast<const void *>(&batch_arg_queue_kernel<64>);
        return reinterpret_cast<const void *>(&batch_arg_queue_kernel<32>);
    }
    if (t.persistent) {
        if (t.tile_w == 16) return reinterpret_cast<const void *>(&batch_persistent_kernel<16, kWalkFirst, kWalkSteps>);
        if (t.tile_w == 64) return reinterpret_cast<const void *>(&batch_persistent_kernel<64, kWalkFirst, kWalkSteps>);
        return reinterpret_cast<const void *>(&batch_persistent_kernel<32, kWalkFirst, kWalkSteps>);
    }
    return args ? width_instance<ArgKernel>(t.tile_w, wf, wb) : width_instance<TableKernel>(t.tile_w, wf, wb);
}

// Workgroups a launch of the plan's tuning uses.
int64_t plan_grid(const rbsm_plan *p) {
    if (!p->tune.persistent) return p->blocks;
    const size_t lds = (size_t)p->tune.lds_cap * sizeof(float);
    return std::min<int64_t>(p->blocks, resident_groups(batch_instance(p->tune, p->use_args), lds));
}

// One batched pass: the RPCF jobs' box-filter kernels, then the tile pass
// over every tile of the other jobs (tables in device memory).
void launch_tables(const rbsm_tuning &tune, const JobDev *jobs, const uint16_t *bj, const BatchArgs *bargs,
                   int *counters, int64_t tiles, int64_t grid, const rbsm_job *host_jobs,
                   const std::vector<int32_t> &rpcf, hipStream_t stream) {
    for (const int32_t j : rpcf) {
        const rbsm_job &J = host_jobs[j];
        if (J.n == 0) continue;
        MapView mv;
        mv.t = J.shadow_map;
        mv.pitch = J.params.pitch;
        mv.W = J.params.width;
        mv.H = J.params.height;
        launch_rpcf(mv, J.frags, J.n, J.params.view_width, J.params.depth_bias, J.params.max_dist,
                    J.params.kernel_radius, static_cast<float *>(J.out), stream);
    }
    if (tiles == 0) return;
    const size_t lds = (size_t)tune.lds_cap * sizeof(float);
    const void *k = batch_instance(tune, bargs != nullptr);
    int apron = tune.apron, cap = tune.lds_cap, chunk = tune.xcd_chunk;
    if (tune.persistent && bargs) {
        int n_tiles = (int)tiles;  // below 2^24
        void *args[] = {(void *)bargs, (void *)&n_tiles, (void *)&apron, (void *)&cap, (void *)&chunk, (void *)&counters};
        (void)hipLaunchKernel(k, dim3((unsigned)grid), dim3(kT), args, lds, stream);
    } else if (!tune.persistent && bargs) {
        void *args[] = {(void *)bargs, (void *)&apron, (void *)&cap, (void *)&chunk};
        (void)hipLaunchKernel(k, dim3((unsigned)tiles), dim3(kT), args, lds, stream);
    } else if (!tune.persistent) {
        void *args[] = {(void *)&jobs, (void *)&bj, (void *)&apron, (void *)&cap, (void *)&chunk};
        (void)hipLaunchKernel(k, dim3((unsigned)tiles), dim3(kT), args, lds, stream);
    } else {
        void *args[] = {(void *)&jobs, (void *)&bj, (void *)&tiles, (void *)&apron, (void *)&cap};
        (void)hipLaunchKernel(k, dim3((unsigned)grid), dim3(kT), args, lds, stream);
    }
}

void launch_batch(const rbsm_plan *p, hipStream_t stream) {
    launch_tables(p->tune, p->d_jobs, p->d_block_job, p->use_args ? &p->args : nullptr, p->d_counters, p->blocks,
                  p->grid, p->jobs.data(), p->rpcf_jobs, stream);
}

// ---------------------------------------------------------------------------
// Batched pass without allocation: its job table and block -> job map live in
// one file-scope device array per GPU (shared by every call on that GPU).
// ---------------------------------------------------------------------------

constexpr size_t kScratchBytes = (size_t)4 << 20;                      // 4 MiB per GPU
constexpr int kScratchJobs = 4096;                                      // job records
constexpr size_t kScratchJobBytes = (size_t)kScratchJobs * sizeof(JobDev);
constexpr int64_t kScratchTiles = (int64_t)((kScratchBytes - kScratchJobBytes) / sizeof(uint16_t));
static_assert(kScratchJobBytes % 256 == 0, "the block map starts 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy of the array at its own address; the
// array's name in host code is not that address).
int scratch_address(const char *fn, void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(RBSM_ERR_HIP, "%s: no current device (or an index beyond 63)", fn);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(RBSM_ERR_HIP, "%s: could not look up the scratch array's device address", fn);
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RBSM_OK;
}

// Job records travel to the scratch table in kernel arguments (copied at
// launch, so the caller's host memory may go at once, and capturable).
constexpr int kChunkJobs = 32;
struct JobChunk {
    int32_t first, count;
    JobDev jobs[kChunkJobs];
};

__global__ __launch_bounds__(64) void upload_jobs_kernel(const JobChunk c, JobDev *table) {
    const int k = threadIdx.x;
    if (k < c.count) table[c.first + k] = c.jobs[k];
}

// block_job[g] = the last job whose first tile is <= g (jobs without tiles
// share their first tile with the next job, which the search prefers).
__global__ __launch_bounds__(256) void block_job_kernel(const JobDev *__restrict__ jobs, int n_jobs, int64_t tiles,
                                                        uint16_t *__restrict__ bj) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= tiles) return;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_base <= g) lo = mid;
        else hi = mid - 1;
    }
    bj[g] = (uint16_t)lo;
}

// Autotuner cache: the chosen tuning per (device, job mix).  The key names
// the device (architecture and CU count) and hashes every job's layout
// (fragment count, view width, map size and pitch, MAXDIST, mode) -- what
// the kernels' speed depends on, not the data.
std::mutex g_tune_mu;
std::map<std::string, rbsm_tuning> g_tune_cache;

std::string tune_key(const rbsm_plan *p) {
    hipDeviceProp_t prop{};
    char dev[96] = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess)
        snprintf(dev, sizeof(dev), "%s-cu%d", prop.gcnArchName, prop.multiProcessorCount);
    for (char *c = dev; *c; ++c)
        if (*c == ' ' || *c == ':') *c = '_';
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the job layout
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)((v >> (8 * b)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    mix((int64_t)p->jobs.size());
    for (const rbsm_job &J : p->jobs) {
        mix(J.n);
        mix(J.params.view_width);
        mix(J.params.width);
        mix(J.params.height);
        mix(J.params.pitch);
        mix(J.params.max_dist);
        mix(J.params.kernel_radius);
        mix(J.mode);
    }
    char key[160];
    snprintf(key, sizeof(key), "%s/%016llx", dev, (unsigned long long)h);
    return key;
}

bool tune_cache_get(const std::string &key, rbsm_tuning *t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) return false;
    *t = it->second;
    return true;
}

void tune_cache_put(const std::string &key, const rbsm_tuning &t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = t;
}

}  // namespace

#include "serve.hpp"

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
        launch_rpcf(mv, frags, n, p->view_width, p->depth_bias, p->max_dist, r, out_vis, stream);
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
    t.persistent = kDefaultTile.persistent;
    t.walk_first = kWalkFirst;
    t.walk_block = kWalkSteps;
    t.xcd_chunk = kDefaultTile.chunk_log2;
    return t;
}

int rbsm_pass_tuned(int32_t mode, const float *shadow_map, const float *frags, int64_t n, const rbsm_params *p,
                    const rbsm_tuning *tune, void *out, hipStream_t stream) {
    if (mode != 0 && mode != 1) return fail(RBSM_ERR_INVALID_ARG, "rbsm_pass_tuned: mode must be 0 or 1");
    if (!tuning_ok(tune)) return fail(RBSM_ERR_INVALID_ARG, "rbsm_pass_tuned: invalid tuning");
    if ((tune->walk_first != 0 && tune->walk_first != kWalkFirst) ||
        (tune->walk_block != 0 && tune->walk_block != kWalkSteps))
        return fail(RBSM_ERR_INVALID_ARG, "rbsm_pass_tuned: walk_first and walk_block must be 0 or the defaults");
    MapView mv;
    const int st = validate("rbsm_pass_tuned", shadow_map, frags, n, p, out, mode == 0 ? 1 : 4, false, &mv);
    if (st != RBSM_OK) return st;
    if (n == 0) return RBSM_OK;
    const TileConfig cfg{tune->tile_w, tune->apron, tune->lds_cap, tune->persistent, tune->xcd_chunk};
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
    if (!p->tune.walk_first) p->tune.walk_first = kWalkFirst;
    if (!p->tune.walk_block) p->tune.walk_block = kWalkSteps;
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
    const bool had_graph = plan->exec != nullptr;
    const int st = build_tables(plan, jobs, n_jobs, true);
    if (st != RBSM_OK || !had_graph) return st;
    // a captured graph holds the launches' arguments (job records, RPCF job
    // pointers): capture again, on a stream of the library's own
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        drop_graph(plan);
        return fail(RBSM_ERR_HIP, "rbsm_plan_update: could not create a stream to capture the plan again");
    }
    const int cst = rbsm_plan_capture(plan, s);
    (void)hipStreamDestroy(s);
    return cst;
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
    rbsm_tuning t = *tune;
    if (!t.walk_first) t.walk_first = kWalkFirst;
    if (!t.walk_block) t.walk_block = kWalkSteps;
    if (t.tile_w != plan->tune.tile_w) {
        const rbsm_tuning old = plan->tune;
        plan->tune = t;
        const std::vector<rbsm_job> jobs = plan->jobs;
        const int st = build_tables(plan, jobs.data(), (int32_t)jobs.size(), false);
        if (st != RBSM_OK) {
            plan->tune = old;
            plan->grid = plan_grid(plan);
            return st;
        }
    }
    plan->tune = t;
    plan->grid = plan_grid(plan);
    return RBSM_OK;
}

int rbsm_plan_get_tuning(const rbsm_plan *plan, rbsm_tuning *tune) {
    if (!plan || !tune) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_get_tuning: null argument");
    *tune = plan->tune;
    return RBSM_OK;
}

int rbsm_plan_autotune(rbsm_plan *plan, hipStream_t stream, int32_t reps, int32_t flags, rbsm_tuning *chosen) {
    if (!plan || reps < 1 || (flags & ~1) != 0) return fail(RBSM_ERR_INVALID_ARG, "rbsm_plan_autotune: invalid argument");
    drop_graph(plan);
    const std::string key = tune_key(plan);
    rbsm_tuning best = plan->tune;
    if (!(flags & 1) && tune_cache_get(key, &best)) {
        const int st = rbsm_plan_set_tuning(plan, &best);
        if (st == RBSM_OK && chosen) *chosen = plan->tune;
        return st;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RBSM_ERR_HIP, "rbsm_plan_autotune: could not create events");
    float best_ms = 1e30f;
    int status = RBSM_OK;
    // time one candidate: a warm-up launch, then reps launches between events
    constexpr float kTuneMargin = 0.02f;
    auto trial = [&](const rbsm_tuning &cand) {
        if (status != RBSM_OK) return;
        if ((status = rbsm_plan_set_tuning(plan, &cand)) != RBSM_OK) return;
        launch_batch(plan, stream);
        (void)hipEventRecord(e0, stream);
        for (int r = 0; r < reps; ++r) launch_batch(plan, stream);
        (void)hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) {
            status = fail(RBSM_ERR_HIP, "rbsm_plan_autotune: a timed launch failed");
            return;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        // a candidate replaces the best only when it is faster by more than
        // kTuneMargin: near-ties keep the earlier (search-order) choice, so
        // timing noise does not flip the tuning from run to run
        if (ms < best_ms * (1.0f - kTuneMargin)) {
            best_ms = ms;
            best = plan->tune;
        }
    };
    // coordinate search: tile shape and schedule, then (one workgroup per
    // tile) how tiles are dealt to XCDs, then LDS capacity, then apron, then
    // the walk blocking
    rbsm_tuning base = rbsm_default_tuning();
    for (int tw : {16, 32, 64})
        for (int per : {0, 1}) {
            rbsm_tuning c = base;
            c.tile_w = tw;
            c.persistent = per;
            trial(c);
        }
    base = best;
    if (!base.persistent || plan->use_args)  // the table-driven persistent loop has its own order
        for (int chunk : {3, 5, 7}) {
            rbsm_tuning c = base;
            c.xcd_chunk = chunk;
            trial(c);
        }
    base = best;
    for (int cap : {0, 1536, 3072, 4096}) {
        rbsm_tuning c = base;
        c.lds_cap = cap;
        trial(c);
    }
    base = best;
    if (base.lds_cap != 0) {  // the apron matters only where tiles are staged
        rbsm_tuning c = base;
        c.apron = base.apron == 1 ? 2 : 1;
        trial(c);
    }
    base = best;
    if (!base.persistent)
        for (int wf : {1, 2, 4})
            for (int wb : {4, 8}) {
                if (wf == base.walk_first && wb == base.walk_block) continue;
                rbsm_tuning c = base;
                c.walk_first = wf;
                c.walk_block = wb;
                trial(c);
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != RBSM_OK) return status;
    if ((status = rbsm_plan_set_tuning(plan, &best)) != RBSM_OK) return status;
    tune_cache_put(key, plan->tune);
    if (chosen) *chosen = plan->tune;
    return RBSM_OK;
}

int rbsm_tune_cache_save(const char *path) {
    if (!path) return fail(RBSM_ERR_INVALID_ARG, "rbsm_tune_cache_save: path is null");
    FILE *f = fopen(path, "w");
    if (!f) return fail(RBSM_ERR_INVALID_ARG, "rbsm_tune_cache_save: cannot open %s", path);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        fprintf(f, "# rbsm tuning cache v2: key tile_w apron lds_cap persistent walk_first walk_block xcd_chunk\n");
        for (const auto &kv : g_tune_cache) {
            const rbsm_tuning &t = kv.second;
            fprintf(f, "%s %d %d %d %d %d %d %d\n", kv.first.c_str(), t.tile_w, t.apron, t.lds_cap, t.persistent,
                    t.walk_first, t.walk_block, t.xcd_chunk);
        }
    }
    const bool ok = fclose(f) == 0;
    return ok ? RBSM_OK : fail(RBSM_ERR_INVALID_ARG, "rbsm_tune_cache_save: write failed for %s", path);
}

int rbsm_tune_cache_load(const char *path) {
    if (!path) return fail(RBSM_ERR_INVALID_ARG, "rbsm_tune_cache_load: path is null");
    FILE *f = fopen(path, "r");
    if (!f) return fail(RBSM_ERR_INVALID_ARG, "rbsm_tune_cache_load: cannot open %s", path);
    char line[512];
    int loaded = 0, status = RBSM_OK;
    while (fgets(line, sizeof(line), f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        char key[256];
        rbsm_tuning t{};
        if (sscanf(line, "%255s %d %d %d %d %d %d %d", key, &t.tile_w, &t.apron, &t.lds_cap, &t.persistent,
                   &t.walk_first, &t.walk_block, &t.xcd_chunk) != 8 ||
            !tuning_ok(&t)) {
            status = fail(RBSM_ERR_INVALID_ARG, "rbsm_tune_cache_load: malformed entry in %s", path);
            break;
        }
        tune_cache_put(key, t);
        ++loaded;
    }
    fclose(f);
    return status == RBSM_OK ? loaded : status;
}

void rbsm_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
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

int rbsm_rasterize(const rbsm_prim *prims, int32_t n_prims, double r0, double ru, double rv, int32_t width,
                   int32_t height, int64_t pitch, float *shadow_map, hipStream_t stream) {
    const char *fn = "rbsm_rasterize";
    if (width < 1 || height < 1 || width > 65536 || height > 65536)
        return fail(RBSM_ERR_INVALID_ARG, "%s: width and height must be in 1..65536", fn);
    if (pitch < width) return fail(RBSM_ERR_INVALID_ARG, "%s: pitch < width", fn);
    if (n_prims < 0) return fail(RBSM_ERR_INVALID_ARG, "%s: n_prims < 0", fn);
    if (!shadow_map || (n_prims > 0 && !prims)) return fail(RBSM_ERR_INVALID_ARG, "%s: null array pointer", fn);
    const size_t map_bytes = ((size_t)(height - 1) * (size_t)pitch + (size_t)width) * 4u;
    if (n_prims > 0 && overlaps(shadow_map, map_bytes, prims, (size_t)n_prims * sizeof(rbsm_prim)))
        return fail(RBSM_ERR_INVALID_ARG, "%s: shadow_map overlaps prims", fn);
    launch_raster(prims, n_prims, r0, ru, rv, width, height, pitch, shadow_map, stream);
    return launched(fn);
}

int rbsm_composite(int64_t n, int32_t n_lights, const void *const *vis, const int32_t *modes, const float *weights,
                   float *out, hipStream_t stream) {
    const char *fn = "rbsm_composite";
    if (n < 0 || n > (int64_t)INT32_MAX) return fail(RBSM_ERR_INVALID_ARG, "%s: n must be in 0..2^31-1", fn);
    if (n_lights < 1 || n_lights > rbsm::kMaxLights) return fail(RBSM_ERR_INVALID_ARG, "%s: n_lights must be 1..8", fn);
    if (!vis || !modes || !weights) return fail(RBSM_ERR_INVALID_ARG, "%s: null host array", fn);
    if (n == 0) return RBSM_OK;
    if (!out) return fail(RBSM_ERR_INVALID_ARG, "%s: out is null", fn);
    rbsm::CompJob J{};
    J.n_lights = n_lights;
    J.n = n;
    J.out = out;
    for (int l = 0; l < n_lights; ++l) {
        if (modes[l] != 0 && modes[l] != 1) return fail(RBSM_ERR_INVALID_ARG, "%s: modes must be 0 or 1", fn);
        if (!vis[l]) return fail(RBSM_ERR_INVALID_ARG, "%s: null visibility pointer", fn);
        if (overlaps(out, (size_t)n * 4u, vis[l], (size_t)n * (modes[l] == 0 ? 1u : 4u)))
            return fail(RBSM_ERR_INVALID_ARG, "%s: out overlaps an input", fn);
        J.vis[l] = vis[l];
        J.w[l] = weights[l];
        J.hard[l] = modes[l] == 0;
    }
    hipLaunchKernelGGL(rbsm::composite_kernel, dim3((unsigned)rbsm::composite_blocks(n)), dim3(rbsm::kCompT), 0,
                       stream, J);
    return launched(fn);
}

int rbsm_engine_create(int64_t hbm_budget_bytes, int32_t max_inflight, rbsm_engine **engine) {
    const char *fn = "rbsm_engine_create";
    if (!engine) return fail(RBSM_ERR_INVALID_ARG, "%s: engine is null", fn);
    *engine = nullptr;
    if (hbm_budget_bytes < 4096) return fail(RBSM_ERR_INVALID_ARG, "%s: budget below 4096 bytes", fn);
    if (max_inflight < 1 || max_inflight > 4096) return fail(RBSM_ERR_INVALID_ARG, "%s: max_inflight must be 1..4096", fn);
    rbsm_engine *E = new (std::nothrow) rbsm_engine;
    if (!E) return fail(RBSM_ERR_INVALID_ARG, "%s: out of host memory", fn);
    E->max_inflight = max_inflight;
    E->budget = hbm_budget_bytes;
    hipError_t e = hipGetDevice(&E->device);
    if (e == hipSuccess) e = hipMalloc(&E->d_arena, (size_t)hbm_budget_bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->s_compute, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->s_copy, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->s_upload, hipStreamNonBlocking);
    for (int s = 0; s < rbsm::kServeSlots && e == hipSuccess; ++s) {
        Slot &S = E->slots[s];
        e = hipEventCreate(&S.compute_start);
        if (e == hipSuccess) e = hipEventCreate(&S.compute_done);
    }
    if (e != hipSuccess) {
        rbsm_engine_destroy(E);
        return fail(RBSM_ERR_HIP, "%s: could not allocate the arena, streams or events", fn);
    }
    E->arena.reset(hbm_budget_bytes);
    E->stats.arena_bytes = hbm_budget_bytes;
    E->worker = std::thread([E] { E->run(); });
    *engine = E;
    return RBSM_OK;
}

int rbsm_engine_add_light(rbsm_engine *E, const float *shadow_map, int32_t width, int32_t height, int64_t pitch,
                          int32_t *light_id) {
    const char *fn = "rbsm_engine_add_light";
    if (!E || !shadow_map || !light_id) return fail(RBSM_ERR_INVALID_ARG, "%s: null argument", fn);
    if (width < 1 || height < 1 || width > 65536 || height > 65536 || pitch < width)
        return fail(RBSM_ERR_INVALID_ARG, "%s: invalid map size or pitch", fn);
    std::lock_guard<std::mutex> lk(E->mu);
    MapView mv;
    mv.t = shadow_map;
    mv.pitch = pitch;
    mv.W = width;
    mv.H = height;
    E->lights.push_back(mv);
    *light_id = (int32_t)E->lights.size() - 1;
    return RBSM_OK;
}

int rbsm_engine_submit(rbsm_engine *E, const rbsm_request *q, int64_t *ticket) {
    const char *fn = "rbsm_engine_submit";
    if (!E || !q || !ticket) return fail(RBSM_ERR_INVALID_ARG, "%s: null argument", fn);
    if (q->n < 0 || q->n > (int64_t)INT32_MAX) return fail(RBSM_ERR_INVALID_ARG, "%s: n must be in 0..2^31-1", fn);
    if (q->view_width < 0) return fail(RBSM_ERR_INVALID_ARG, "%s: view_width < 0", fn);
    if (q->n_lights < 1 || q->n_lights > rbsm::kMaxLights)
        return fail(RBSM_ERR_INVALID_ARG, "%s: n_lights must be 1..8", fn);
    EngineReq *R = new (std::nothrow) EngineReq;
    if (!R) return fail(RBSM_ERR_INVALID_ARG, "%s: out of host memory", fn);
    R->req = *q;
    for (int l = 0; l < q->n_lights; ++l) {
        R->direct_out[l] = q->n > 0 && is_device_memory(q->lights[l].out, E->device);
        R->host_frags[l] = q->n > 0 && q->lights[l].frags && !is_device_memory(q->lights[l].frags, E->device);
        R->uploads = R->uploads || R->host_frags[l];
    }
    R->direct_comp = q->n > 0 && is_device_memory(q->composite, E->device);
    R->bytes = request_bytes(*R);
    R->work = request_work(*R);
    if (R->work > E->budget) {
        delete R;
        return fail(RBSM_ERR_INVALID_ARG, "%s: the request's fragments and results alone exceed the HBM budget", fn);
    }
    {
        std::lock_guard<std::mutex> lk(E->mu);
        for (int l = 0; l < q->n_lights; ++l) {
            const rbsm_request_light &L = q->lights[l];
            const char *bad = nullptr;
            if (L.light < 0 || L.light >= (int32_t)E->lights.size()) bad = "unknown light";
            else if (L.mode != 0 && L.mode != 1) bad = "mode must be 0 or 1";
            else if (L.max_dist < 1 || L.max_dist > 64) bad = "max_dist must be in 1..64";
            else if (L.kernel_radius < 0 || L.kernel_radius > 32) bad = "kernel_radius must be in 0..32";
            else if (L.mode == 0 && L.kernel_radius != 0) bad = "kernel_radius must be 0 in hard mode";
            else if (q->n > 0 && !L.frags) bad = "null fragments";
            if (bad) {
                delete R;
                return fail(RBSM_ERR_INVALID_ARG, "rbsm_engine_submit: %s", bad);
            }
            R->maps[l] = E->lights[L.light];
        }
        // results written in place must not overlap any input of the request
        for (int a = 0; a < q->n_lights + 1; ++a) {
            const bool is_comp = a == q->n_lights;
            if (is_comp ? !R->direct_comp : !R->direct_out[a]) continue;
            const void *dst = is_comp ? (const void *)q->composite : q->lights[a].out;
            const size_t db = (size_t)q->n * (is_comp || q->lights[a].mode != 0 ? 4u : 1u);
            for (int b = 0; b < q->n_lights; ++b) {
                const MapView &mv = R->maps[b];
                const size_t mb = ((size_t)(mv.H - 1) * (size_t)mv.pitch + (size_t)mv.W) * 4u;
                bool bad = overlaps(dst, db, q->lights[b].frags, (size_t)q->n * 12u) || overlaps(dst, db, mv.t, mb);
                if (!is_comp && b != a && R->direct_out[b])
                    bad = bad || overlaps(dst, db, q->lights[b].out, (size_t)q->n * (q->lights[b].mode == 0 ? 1u : 4u));
                if (is_comp && R->direct_out[b])
                    bad = bad || overlaps(dst, db, q->lights[b].out, (size_t)q->n * (q->lights[b].mode == 0 ? 1u : 4u));
                if (bad) {
                    delete R;
                    return fail(RBSM_ERR_INVALID_ARG, "rbsm_engine_submit: a device result buffer overlaps an input",
                                nullptr);
                }
            }
        }
        if (!E->error.empty()) {
            delete R;
            return fail(RBSM_ERR_HIP, "rbsm_engine_submit: engine failed earlier: %s", E->error.c_str());
        }
    }
    // events: results done, uploads done, and the caller's stream at submit
    // (the engine's kernels wait for everything enqueued on it so far)
    hipError_t ev = hipEventCreateWithFlags(&R->done, hipEventDisableTiming);
    if (ev == hipSuccess) ev = hipEventCreateWithFlags(&R->ready, hipEventDisableTiming);
    if (ev == hipSuccess && R->uploads) ev = hipEventCreateWithFlags(&R->uploaded, hipEventDisableTiming);
    if (ev == hipSuccess) ev = hipEventRecord(R->ready, q->stream);
    if (ev != hipSuccess) {
        (void)hipGetLastError();
        if (R->done) (void)hipEventDestroy(R->done);
        if (R->ready) (void)hipEventDestroy(R->ready);
        if (R->uploaded) (void)hipEventDestroy(R->uploaded);
        delete R;
        return fail(RBSM_ERR_HIP, "%s: could not create or record the request's events", fn);
    }
    std::lock_guard<std::mutex> lk(E->mu);
    R->t_submit = Clock::now();
    R->ticket = E->next_ticket++;
    E->tickets[R->ticket] = R;
    E->queue.push_back(R);
    E->stats.submitted += 1;
    E->stats.queued += 1;
    *ticket = R->ticket;
    E->cv_work.notify_one();
    return RBSM_OK;
}

int rbsm_engine_wait(rbsm_engine *E, int64_t ticket, int32_t timeout_ms, double *latency_ms) {
    const char *fn = "rbsm_engine_wait";
    if (!E) return fail(RBSM_ERR_INVALID_ARG, "%s: engine is null", fn);
    std::unique_lock<std::mutex> lk(E->mu);
    auto it = E->tickets.find(ticket);
    if (it == E->tickets.end()) return fail(RBSM_ERR_INVALID_ARG, "%s: unknown ticket", fn);
    EngineReq *R = it->second;
    auto ready = [&] { return R->status != 0; };
    if (timeout_ms < 0) E->cv_done.wait(lk, ready);
    else if (!E->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) return 0;
    const int status = R->status;
    const double ms = std::chrono::duration<double, std::milli>(R->t_done - R->t_submit).count();
    E->tickets.erase(it);
    const std::string err = E->error;
    lk.unlock();
    (void)hipEventDestroy(R->done);
    (void)hipEventDestroy(R->ready);
    if (R->uploaded) (void)hipEventDestroy(R->uploaded);
    delete R;
    if (status < 0) return fail(RBSM_ERR_HIP, "rbsm_engine_wait: %s", err.c_str());
    if (latency_ms) *latency_ms = ms;
    return 1;
}

int rbsm_engine_abort(rbsm_engine *E, const char *reason) {
    if (!E) return fail(RBSM_ERR_INVALID_ARG, "rbsm_engine_abort: engine is null");
    {
        std::lock_guard<std::mutex> lk(E->mu);
        E->abort_reason = std::string("engine aborted: ") + (reason ? reason : "by the caller");
    }
    E->cv_work.notify_all();
    return RBSM_OK;
}

int rbsm_engine_get_stats(rbsm_engine *E, rbsm_engine_stats *stats) {
    if (!E || !stats) return fail(RBSM_ERR_INVALID_ARG, "rbsm_engine_get_stats: null argument");
    std::lock_guard<std::mutex> lk(E->mu);
    *stats = E->stats;
    return RBSM_OK;
}

void rbsm_engine_destroy(rbsm_engine *E) {
    if (!E) return;
    if (E->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(E->mu);
            E->stop = true;
        }
        E->cv_work.notify_all();
        E->worker.join();
    }
    if (E->s_upload) (void)hipStreamSynchronize(E->s_upload);
    if (E->s_compute) (void)hipStreamSynchronize(E->s_compute);
    if (E->s_copy) (void)hipStreamSynchronize(E->s_copy);
    for (auto &kv : E->tickets) {
        (void)hipEventDestroy(kv.second->done);
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
        if (kv.second->uploaded) (void)hipEventDestroy(kv.second->uploaded);
        delete kv.second;
    }
    for (Slot &S : E->slots) {
        if (S.compute_start) (void)hipEventDestroy(S.compute_start);
        if (S.compute_done) (void)hipEventDestroy(S.compute_done);
    }
    if (E->s_compute) (void)hipStreamDestroy(E->s_compute);
    if (E->s_copy) (void)hipStreamDestroy(E->s_copy);
    if (E->s_upload) (void)hipStreamDestroy(E->s_upload);
    if (E->d_arena) (void)hipFree(E->d_arena);
    delete E;
}

int rbsm_batch_launch_noalloc(const rbsm_job *jobs, int32_t n_jobs, const rbsm_tuning *tune, hipStream_t stream) {
    const char *fn = "rbsm_batch_launch_noalloc";
    if (tune && !tuning_ok(tune)) return fail(RBSM_ERR_INVALID_ARG, "%s: invalid tuning", fn);
    rbsm_tuning t = tune ? *tune : rbsm_default_tuning();
    if (!t.walk_first) t.walk_first = kWalkFirst;
    if (!t.walk_block) t.walk_block = kWalkSteps;
    if (n_jobs > kScratchJobs) return fail(RBSM_ERR_INVALID_ARG, "%s: at most 4096 jobs per call", fn);
    HostTables T;
    int st = make_tables(fn, jobs, n_jobs, t.tile_w, nullptr, false, false, T);
    if (st != RBSM_OK) return st;
    if (T.tiles > kScratchTiles)
        return fail(RBSM_ERR_INVALID_ARG, "%s: the jobs need more than 1,916,928 screen tiles", fn);
    void *base = nullptr;
    if ((st = scratch_address(fn, &base)) != RBSM_OK) return st;
    JobDev *d_jobs = static_cast<JobDev *>(base);
    uint16_t *d_bj = reinterpret_cast<uint16_t *>(static_cast<char *>(base) + kScratchJobBytes);
    for (int32_t first = 0; first < n_jobs; first += kChunkJobs) {
        JobChunk c{};
        c.first = first;
        c.count = std::min(kChunkJobs, n_jobs - first);
        for (int k = 0; k < c.count; ++k) c.jobs[k] = T.dev[first + k];
        hipLaunchKernelGGL(upload_jobs_kernel, dim3(1), dim3(64), 0, stream, c, d_jobs);
    }
    if (T.tiles > 0)
        hipLaunchKernelGGL(block_job_kernel, dim3((unsigned)((T.tiles + 255) / 256)), dim3(256), 0, stream,
                           (const JobDev *)d_jobs, n_jobs, T.tiles, d_bj);
    const size_t lds = (size_t)t.lds_cap * sizeof(float);
    const int64_t grid =
        t.persistent ? std::min<int64_t>(T.tiles, resident_groups(batch_instance(t, false), lds)) : T.tiles;
    launch_tables(t, d_jobs, d_bj, nullptr, nullptr, T.tiles, grid, jobs, T.rpcf, stream);
    return launched(fn);
}

const char *rbsm_last_error(void) { return g_err; }

int32_t rbsm_abi_version(void) { return 103; }

}  // extern "C"
