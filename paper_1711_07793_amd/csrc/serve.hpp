// Serving form and multi-light compositing.  Included once, by rbsm.hip, after
// the argument checks and job layout it uses.
//
// Compositing: a view lit by several lights gets one shadow value per
// fragment, the weighted sum of its per-light visibilities (Listing 1 scales a
// light's contribution by its visibility; the paper does not define how
// lights combine, so the weights are the caller's per-light intensities),
// summed in light order in binary32, product then sum.
//
// Engine: a native scheduler thread over a fixed HBM budget (one device arena
// allocated at creation).  Requests (a view's fragments for 1..8 resident
// lights) are admitted first-come first-served while arena space and an
// in-flight slot are free; every scheduling step launches ONE pass over the
// jobs of all admitted requests (the same tile code as the plain entry points,
// so each per-light result is bitwise that of rbsm_visibility /
// rsmss_visibility), then RPCF jobs, then one compositing launch.  Result
// buffers in device memory are written in place; host buffers are staged in
// the arena and copied back on a second stream while the next step computes.
// Requests that arrive while others run join the next step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.hpp"
#include "rbsm.h"
#include "tile_pass.hpp"

namespace rbsm {

constexpr int kMaxLights = 8;
constexpr int kServeMaxJobs = 256;   // (request, light) jobs per scheduling step
constexpr int kServeMaxReqs = 64;    // requests per scheduling step
constexpr int kServeSlots = 2;       // steps whose compute may be pending
constexpr int kArgJobs = 40;         // tile jobs per launch, passed in the kernel arguments
constexpr int kArgComp = 20;         // composites per launch, passed in the kernel arguments
constexpr int kServeTileW = 64;      // tile width of the merged jobs (as in the batched autotuner's choice)
constexpr int kServeChunkLog2 = 5;   // merged jobs' tiles dealt to XCDs in chunks of 32 (balances XCDs)

// One view's composite: out[k] = sum_l w[l] * vis_l[k].
struct CompJob {
    const void *vis[kMaxLights];
    float w[kMaxLights];
    int32_t hard[kMaxLights];  // 1: uint8 mask, 0: float visibility
    int32_t n_lights;
    int64_t n;
    float *out;
};

constexpr int kCompT = 256, kCompF = 4;  // threads, fragments per thread

__device__ __forceinline__ float comp_value(const CompJob &J, int l, int64_t k) {
    return J.hard[l] ? (float)static_cast<const uint8_t *>(J.vis[l])[k] : static_cast<const float *>(J.vis[l])[k];
}

// Each thread owns 4 consecutive fragments.  When every buffer of the job is
// aligned for it (masks to 4 bytes, visibilities and the output to 16), each
// light is one 4- or 16-byte load and the result one 16-byte store; otherwise,
// and at a ragged end, fragment by fragment.  Either way a fragment's sum runs
// over the lights in order with the same operations.
__device__ __forceinline__ void composite_range(const CompJob &J, int64_t block_first) {
    const int64_t k = block_first + 4 * (int64_t)threadIdx.x;
    if (k >= J.n) return;
    bool vec = (((uintptr_t)J.out) & 15u) == 0;
    for (int l = 0; l < J.n_lights; ++l) vec = vec && (((uintptr_t)J.vis[l]) & (J.hard[l] ? 3u : 15u)) == 0;
    if (vec && k + 3 < J.n) {
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int l = 0; l < J.n_lights; ++l) {
            float v[4];
            if (J.hard[l]) {
                const uint32_t b = *(const uint32_t *)(static_cast<const uint8_t *>(J.vis[l]) + k);
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = (float)((b >> (8 * e)) & 255u);
            } else {
                const float4 f = *(const float4 *)(static_cast<const float *>(J.vis[l]) + k);
                v[0] = f.x;
                v[1] = f.y;
                v[2] = f.z;
                v[3] = f.w;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = acc[e] + J.w[l] * v[e];
        }
        *(float4 *)(J.out + k) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        return;
    }
    for (int e = 0; e < 4 && k + e < J.n; ++e) {
        float acc = 0.0f;
        for (int l = 0; l < J.n_lights; ++l) acc = acc + J.w[l] * comp_value(J, l, k + e);
        J.out[k + e] = acc;
    }
}

__global__ __launch_bounds__(kCompT) void composite_kernel(CompJob J) {
    composite_range(J, (int64_t)blockIdx.x * (kCompT * kCompF));
}

inline int64_t composite_blocks(int64_t n) { return (n + kCompT * kCompF - 1) / (kCompT * kCompF); }

// Job tables of one launch travel in the kernel arguments (read with scalar
// loads, no copy of their own); a block finds its job by binary search over
// the jobs' first blocks.
struct CompArgs {
    int32_t n_jobs;
    int64_t first[kArgComp];
    CompJob jobs[kArgComp];
};

struct ServeArgs {
    int32_t n_jobs;
    int64_t first[kArgJobs];
    JobDev jobs[kArgJobs];
};

__device__ __forceinline__ int find_job(const int64_t *first, int n, int64_t g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kCompT) void composite_batch_kernel(const CompArgs a) {
    const int64_t g = blockIdx.x;
    const int j = find_job(a.first, a.n_jobs, g);
    composite_range(a.jobs[j], (g - a.first[j]) * (kCompT * kCompF));
}

// The batched tile pass of a scheduling step, one launch per chunk of jobs of
// either mode: each tile runs the steps of the single-view pass, with its
// occupancy (64 VGPRs, 8 workgroups per CU at the default LDS capacity).  IX
// = int when every job of the launch fits the 32-bit index form (index32).
template <int TW, class IX>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(8, 8))) void serve_kernel(const ServeArgs a,
                                                                                              int apron, int cap) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    const int64_t g = xcd_chunked(blockIdx.x, gridDim.x, kServeChunkLog2);
    const int j = find_job(a.first, a.n_jobs, g);
    const JobDev &J = a.jobs[j];
    process_tile<2, TW, kWalkFirst, kWalkSteps, IX, true>(J.m, J.frags, J.n, J.vw, J.tiles_x, J.bias, J.maxd, apron,
                                                          cap, J.vec_ok, J.out, g - a.first[j], sh, s_tex,
                                                          J.mode == 0);
}

}  // namespace rbsm

// ---------------------------------------------------------------------------
// engine state (host)
// ---------------------------------------------------------------------------

namespace {

using Clock = std::chrono::steady_clock;

struct EngineReq {
    int64_t ticket = 0;
    rbsm_request req{};
    MapView maps[rbsm::kMaxLights]{};
    int64_t off = -1, bytes = 0;         // arena block (staged fragments and results)
    int64_t work = 0;                    // HBM working set counted against the budget
    const float *d_frags[rbsm::kMaxLights]{};  // per-light device fragments (caller's or arena)
    void *d_out[rbsm::kMaxLights]{};     // per-light device results (caller's or arena)
    float *d_comp = nullptr;             // device composite (caller's or arena), or null
    bool direct_out[rbsm::kMaxLights]{}; // the caller's buffer is device memory: written in place
    bool direct_comp = false;
    bool host_frags[rbsm::kMaxLights]{}; // fragments in host memory: uploaded into the arena
    bool uploads = false;                // some fragments are uploaded
    Clock::time_point t_submit, t_done;
    hipEvent_t ready = nullptr;          // recorded on the caller's stream at submit
    hipEvent_t uploaded = nullptr;       // the request's uploads are in the arena
    hipEvent_t done = nullptr;           // every result is in its buffer
    int status = 0;                      // 0 pending, 1 done, < 0 failed
};

struct Slot {
    hipEvent_t compute_start = nullptr, compute_done = nullptr;  // timing events around a step's compute
    bool busy = false;
};

// Arena bytes of a request: every per-light result not written in place, the
// composite when it is staged, and the fragments of lights whose fragments are
// in host memory (uploaded).
int64_t request_bytes(const EngineReq &R) {
    const rbsm_request &r = R.req;
    int64_t b = 0;
    for (int l = 0; l < r.n_lights; ++l) {
        if (!R.direct_out[l]) b += rbsm::Arena::round_up(r.n * (r.lights[l].mode == 0 ? 1 : 4));
        if (R.host_frags[l]) b += rbsm::Arena::round_up(r.n * 12);
    }
    if (r.composite && !R.direct_comp) b += rbsm::Arena::round_up(r.n * 4);
    return b;
}

// HBM working set of a request while it is admitted: its fragments (12 B per
// fragment and light) and its results (1 or 4 B per fragment and light, 4 B
// for the composite), wherever they live.  Admission keeps the sum over
// admitted requests within the budget.
int64_t request_work(const EngineReq &R) {
    const rbsm_request &r = R.req;
    int64_t b = 0;
    for (int l = 0; l < r.n_lights; ++l) b += r.n * (12 + (r.lights[l].mode == 0 ? 1 : 4));
    if (r.composite) b += r.n * 4;
    return b;
}

// Is p device memory of `device` (so kernels may write it in place)?
bool is_device_memory(const void *p, int device) {
    if (!p) return false;
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // pageable host memory reports an error; clear it
        return false;
    }
    return a.type == hipMemoryTypeDevice && a.device == device;
}

}  // namespace

struct rbsm_engine {
    int device = 0;
    char *d_arena = nullptr;
    rbsm::Arena arena;  // worker thread only
    int32_t max_inflight = 1;
    int64_t budget = 0;       // HBM budget of the admitted requests' working sets
    int64_t work = 0;         // their current sum (worker thread only)
    hipStream_t s_compute = nullptr, s_copy = nullptr, s_upload = nullptr;
    Slot slots[rbsm::kServeSlots];

    std::mutex mu;  // guards everything below
    std::condition_variable cv_work, cv_done;
    std::vector<MapView> lights;
    std::deque<EngineReq *> queue;                   // submitted, not admitted
    std::unordered_map<int64_t, EngineReq *> tickets;  // not yet collected by wait()
    int64_t next_ticket = 1;
    bool stop = false;
    std::string error;
    std::string abort_reason;  // set by rbsm_engine_abort, acted on by the worker
    rbsm_engine_stats stats{};

    std::vector<EngineReq *> admitted;  // worker thread only
    std::vector<EngineReq *> inflight;  // worker thread only
    std::thread worker;

    void run();
    bool step_launch();
    void fail_all(const char *what, hipError_t e);
};

namespace {

// A free step slot (at most kServeSlots steps have compute pending), or -1.
int pick_slot(rbsm_engine *E) {
    for (int s = 0; s < rbsm::kServeSlots; ++s)
        if (!E->slots[s].busy) return s;
    return -1;
}

}  // namespace

void rbsm_engine::fail_all(const char *what, hipError_t e) {
    // work already enqueued may still write the callers' buffers (host
    // copies included): let it finish before anyone learns of the failure
    (void)hipStreamSynchronize(s_upload);
    (void)hipStreamSynchronize(s_compute);
    (void)hipStreamSynchronize(s_copy);
    (void)hipGetLastError();
    for (int s = 0; s < rbsm::kServeSlots; ++s) slots[s].busy = false;
    std::lock_guard<std::mutex> lk(mu);
    if (error.empty()) error = e == hipSuccess ? std::string(what) : std::string(what) + ": " + hipGetErrorString(e);
    const Clock::time_point now = Clock::now();
    for (std::vector<EngineReq *> *list : {&admitted, &inflight}) {
        for (auto *r : *list) {
            if (r->bytes > 0 && r->off >= 0) arena.release(r->off, r->bytes);
            r->status = RBSM_ERR_HIP;
            r->t_done = now;
            stats.inflight -= 1;
        }
        list->clear();
    }
    for (auto *r : queue) {
        r->status = RBSM_ERR_HIP;
        r->t_done = now;
        stats.queued -= 1;
    }
    queue.clear();
    work = 0;
    stats.inflight_bytes = 0;
    cv_done.notify_all();
}

bool rbsm_engine::step_launch() {
    const int s = pick_slot(this);
    if (s < 0 || admitted.empty()) return false;
    Slot &S = slots[s];
    std::vector<EngineReq *> batch;
    std::vector<std::pair<EngineReq *, int>> rpcf_jobs, tile_jobs;  // (request, light)
    std::vector<rbsm::CompJob> comps;
    int n_jobs = 0;
    size_t taken = 0;
    for (; taken < admitted.size(); ++taken) {
        EngineReq *R = admitted[taken];
        const rbsm_request &q = R->req;
        if (n_jobs + q.n_lights > rbsm::kServeMaxJobs || (int)batch.size() >= rbsm::kServeMaxReqs) break;
        n_jobs += q.n_lights;
        for (int l = 0; l < q.n_lights; ++l) {
            if (q.lights[l].kernel_radius > 0) rpcf_jobs.push_back({R, l});
            else tile_jobs.push_back({R, l});
        }
        if (R->d_comp && q.n > 0) {
            rbsm::CompJob C{};
            C.n_lights = q.n_lights;
            C.n = q.n;
            C.out = R->d_comp;
            for (int l = 0; l < q.n_lights; ++l) {
                C.vis[l] = R->d_out[l];
                C.w[l] = q.lights[l].weight;
                C.hard[l] = q.lights[l].mode == 0;
            }
            comps.push_back(C);
        }
        batch.push_back(R);
    }
    if (batch.empty()) return false;
    admitted.erase(admitted.begin(), admitted.begin() + taken);

    hipError_t e = hipSuccess;
    // the callers' producer streams and the fragment uploads come first
    for (EngineReq *R : batch) {
        if (e == hipSuccess) e = hipStreamWaitEvent(s_compute, R->ready, 0);
        if (e == hipSuccess && R->uploads) e = hipStreamWaitEvent(s_compute, R->uploaded, 0);
    }
    if (e == hipSuccess) e = hipEventRecord(S.compute_start, s_compute);
    const size_t lds = (size_t)kDefaultTile.cap * sizeof(float);
    // tile jobs of both modes, in chunks that fit the kernel arguments
    {
        const auto &list = tile_jobs;
        for (size_t c0 = 0; c0 < list.size() && e == hipSuccess; c0 += rbsm::kArgJobs) {
            rbsm::ServeArgs A{};
            int64_t tiles = 0;
            bool ix32 = true;
            for (size_t c = c0; c < list.size() && c < c0 + rbsm::kArgJobs; ++c) {
                const EngineReq *R = list[c].first;
                const rbsm_request &q = R->req;
                const rbsm_request_light &L = q.lights[list[c].second];
                const JobLayout lay = job_layout(q.n, q.view_width, rbsm::kServeTileW);
                if (lay.tiles == 0) continue;
                JobDev &D = A.jobs[A.n_jobs];
                D.m = R->maps[list[c].second];
                D.frags = R->d_frags[list[c].second];
                D.out = R->d_out[list[c].second];
                D.n = q.n;
                D.vw = lay.vw;
                D.tiles_x = lay.tiles_x;
                D.tile_base = 0;
                D.bias = L.depth_bias;
                D.maxd = L.max_dist;
                D.mode = L.mode;
                D.vec_ok = ((uintptr_t)D.frags % 16 == 0) && ((uintptr_t)D.out % (L.mode == 0 ? 4 : 16) == 0) &&
                           (lay.vw % 4 == 0);
                ix32 = ix32 && rbsm::index32(q.n, lay.vw, rbsm::kServeTileW);
                A.first[A.n_jobs++] = tiles;
                tiles += lay.tiles;
            }
            if (tiles == 0) continue;
            if (ix32)
                hipLaunchKernelGGL((rbsm::serve_kernel<rbsm::kServeTileW, int>), dim3((unsigned)tiles), dim3(kT), lds,
                                   s_compute, A, kDefaultTile.apron, kDefaultTile.cap);
            else
                hipLaunchKernelGGL((rbsm::serve_kernel<rbsm::kServeTileW, int64_t>), dim3((unsigned)tiles), dim3(kT),
                                   lds, s_compute, A, kDefaultTile.apron, kDefaultTile.cap);
        }
    }
    for (const auto &rj : rpcf_jobs) {
        const rbsm_request &q = rj.first->req;
        const rbsm_request_light &L = q.lights[rj.second];
        if (q.n == 0) continue;
        launch_rpcf(rj.first->maps[rj.second], rj.first->d_frags[rj.second], q.n, q.view_width, L.depth_bias,
                    L.max_dist, L.kernel_radius, static_cast<float *>(rj.first->d_out[rj.second]), s_compute);
    }
    for (size_t c0 = 0; c0 < comps.size(); c0 += rbsm::kArgComp) {
        rbsm::CompArgs A{};
        int64_t blocks = 0;
        for (size_t c = c0; c < comps.size() && c < c0 + rbsm::kArgComp; ++c) {
            A.jobs[A.n_jobs] = comps[c];
            A.first[A.n_jobs++] = blocks;
            blocks += rbsm::composite_blocks(comps[c].n);
        }
        hipLaunchKernelGGL(rbsm::composite_batch_kernel, dim3((unsigned)blocks), dim3(rbsm::kCompT), 0, s_compute, A);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(S.compute_done, s_compute);
    if (e == hipSuccess) e = hipStreamWaitEvent(s_copy, S.compute_done, 0);
    for (EngineReq *R : batch) {
        const rbsm_request &q = R->req;
        for (int l = 0; l < q.n_lights && e == hipSuccess; ++l)
            if (q.lights[l].out && !R->direct_out[l] && q.n > 0)
                e = hipMemcpyAsync(q.lights[l].out, R->d_out[l], (size_t)q.n * (q.lights[l].mode == 0 ? 1 : 4),
                                   hipMemcpyDefault, s_copy);
        if (e == hipSuccess && q.composite && !R->direct_comp && q.n > 0)
            e = hipMemcpyAsync(q.composite, R->d_comp, (size_t)q.n * 4, hipMemcpyDefault, s_copy);
        if (e == hipSuccess) e = hipEventRecord(R->done, s_copy);
        inflight.push_back(R);
    }
    if (e != hipSuccess) {
        fail_all("engine: launch", e);
        return false;
    }
    S.busy = true;
    {
        std::lock_guard<std::mutex> lk(mu);
        stats.launches += 1;
        stats.jobs_launched += n_jobs;
    }
    return true;
}

void rbsm_engine::run() {
    (void)hipSetDevice(device);
    Clock::time_point idle_since{};
    hipError_t upload_error = hipSuccess;
    for (;;) {
        bool progress = false;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (!abort_reason.empty()) {
                const std::string why = abort_reason;
                abort_reason.clear();
                lk.unlock();
                fail_all(why.c_str(), hipSuccess);
                continue;
            }
        }
        // steps whose compute finished free their table slot
        for (int s = 0; s < rbsm::kServeSlots; ++s) {
            if (!slots[s].busy) continue;
            const hipError_t q = hipEventQuery(slots[s].compute_done);
            if (q == hipSuccess) {
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, slots[s].compute_start, slots[s].compute_done);
                slots[s].busy = false;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    stats.gpu_busy_ns += (int64_t)(ms * 1e6);
                }
                progress = true;
            } else if (q != hipErrorNotReady) {
                fail_all("engine: compute", q);
            }
        }
        // finished requests release their arena block
        for (size_t i = 0; i < inflight.size();) {
            EngineReq *R = inflight[i];
            const hipError_t q = hipEventQuery(R->done);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            if (R->bytes > 0) arena.release(R->off, R->bytes);
            work -= R->work;
            std::lock_guard<std::mutex> lk(mu);
            stats.inflight_bytes = work;
            R->t_done = Clock::now();
            R->status = q == hipSuccess ? 1 : RBSM_ERR_HIP;
            if (q != hipSuccess && error.empty()) error = std::string("engine: copy: ") + hipGetErrorString(q);
            stats.completed += 1;
            stats.inflight -= 1;
            stats.fragments_completed += R->req.n * R->req.n_lights;
            inflight[i] = inflight.back();
            inflight.pop_back();
            cv_done.notify_all();
            progress = true;
        }
        // admission: first come, first served, by arena space and slots
        {
            std::lock_guard<std::mutex> lk(mu);
            while (!queue.empty() && (int64_t)(admitted.size() + inflight.size()) < max_inflight) {
                EngineReq *R = queue.front();
                if (work + R->work > budget) break;  // the working sets stay within the HBM budget
                const int64_t off = R->bytes > 0 ? arena.alloc(R->bytes) : 0;  // nothing staged: no block
                if (off < 0) break;
                R->off = off;
                char *p = d_arena + off;
                const int64_t n = R->req.n;
                hipError_t e = hipSuccess;
                for (int l = 0; l < R->req.n_lights; ++l) {
                    if (R->host_frags[l]) {  // uploaded on the upload stream while earlier steps compute
                        R->d_frags[l] = reinterpret_cast<const float *>(p);
                        if (e == hipSuccess)
                            e = hipMemcpyAsync(p, R->req.lights[l].frags, (size_t)n * 12, hipMemcpyHostToDevice,
                                               s_upload);
                        p += rbsm::Arena::round_up(n * 12);
                        stats.uploaded_bytes += n * 12;
                    } else {
                        R->d_frags[l] = R->req.lights[l].frags;
                    }
                    if (R->direct_out[l]) {
                        R->d_out[l] = R->req.lights[l].out;
                        continue;
                    }
                    R->d_out[l] = p;
                    p += rbsm::Arena::round_up(n * (R->req.lights[l].mode == 0 ? 1 : 4));
                }
                R->d_comp = R->direct_comp ? R->req.composite
                                           : (R->req.composite ? reinterpret_cast<float *>(p) : nullptr);
                if (e == hipSuccess && R->uploads) e = hipEventRecord(R->uploaded, s_upload);
                work += R->work;
                stats.inflight_bytes = work;
                stats.inflight_peak_bytes = std::max(stats.inflight_peak_bytes, work);
                queue.pop_front();
                admitted.push_back(R);
                stats.queued -= 1;
                stats.inflight += 1;
                stats.arena_peak_bytes = arena.peak();
                progress = true;
                if (e != hipSuccess) {  // the request holds its block and budget: fail_all releases them
                    upload_error = e;
                    break;
                }
            }
        }
        if (upload_error != hipSuccess) {
            fail_all("engine: fragment upload", upload_error);
            upload_error = hipSuccess;
            continue;
        }
        if (step_launch()) progress = true;
        if (!progress) {
            // with work on the device, poll (yielding the core); idle, sleep
            // until a submission arrives
            if (!admitted.empty() || !inflight.empty()) {
                std::this_thread::yield();
                idle_since = Clock::time_point{};
                continue;
            }
            std::unique_lock<std::mutex> lk(mu);
            if (stop && queue.empty()) break;
            if (!queue.empty() || !abort_reason.empty()) continue;
            // idle: keep polling for a short while (a request arriving now is
            // picked up at once), then sleep until a submission
            const auto now = Clock::now();
            if (idle_since == Clock::time_point{}) idle_since = now;
            if (now - idle_since < std::chrono::microseconds(500)) {
                lk.unlock();
                std::this_thread::yield();
                continue;
            }
            cv_work.wait(lk, [&] { return stop || !queue.empty() || !abort_reason.empty(); });
            idle_since = Clock::time_point{};
        }
    }
}
