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
// rsmss_visibility), then RPCF jobs, then one compositing launch, and copies
// results to the callers' host buffers on a second stream while the next step
// computes.  Requests that arrive while others run join the next step.
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
constexpr int kServeMaxJobs = 256;   // jobs per scheduling step
constexpr int kServeMaxReqs = 64;    // requests per scheduling step
constexpr int kServeSlots = 4;       // table slots (steps whose compute may be pending)
constexpr int kServeComputeAhead = 2;

// One view's composite: out[k] = sum_l w[l] * vis_l[k].
struct CompJob {
    const void *vis[kMaxLights];
    float w[kMaxLights];
    int32_t hard[kMaxLights];  // 1: uint8 mask, 0: float visibility
    int32_t n_lights;
    int64_t n;
    float *out;
    int64_t block_base;  // first block of this job in a batched launch
};

constexpr int kCompT = 256, kCompF = 4;  // threads, fragments per thread

__device__ __forceinline__ void composite_range(const CompJob &J, int64_t first) {
    for (int e = 0; e < kCompF; ++e) {
        const int64_t k = first + (int64_t)e * kCompT;
        if (k >= J.n) return;
        float acc = 0.0f;
        for (int l = 0; l < J.n_lights; ++l) {
            const float v = J.hard[l] ? (float)static_cast<const uint8_t *>(J.vis[l])[k]
                                      : static_cast<const float *>(J.vis[l])[k];
            acc = acc + J.w[l] * v;
        }
        J.out[k] = acc;
    }
}

__global__ __launch_bounds__(kCompT) void composite_kernel(CompJob J) {
    composite_range(J, (int64_t)blockIdx.x * (kCompT * kCompF) + threadIdx.x);
}

// Several composites in one launch; jobs sorted by block_base.
__global__ __launch_bounds__(kCompT) void composite_batch_kernel(const CompJob *__restrict__ jobs, int n_jobs) {
    __shared__ int64_t s_base[kServeMaxReqs];
    for (int t = threadIdx.x; t < n_jobs; t += kCompT) s_base[t] = jobs[t].block_base;
    __syncthreads();
    const int64_t g = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_base[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    const CompJob J = jobs[lo];
    composite_range(J, (g - J.block_base) * (kCompT * kCompF) + threadIdx.x);
}

inline int64_t composite_blocks(int64_t n) { return (n + kCompT * kCompF - 1) / (kCompT * kCompF); }

// The batched tile pass of a scheduling step: like batch_kernel, but the
// block -> job lookup is a binary search over the jobs' first tiles (staged
// in LDS), so a step needs no per-tile table.
template <int TW>
__global__ __launch_bounds__(kT) void serve_kernel(const JobDev *__restrict__ jobs, int n_jobs, int apron, int cap) {
    extern __shared__ float s_tex[];
    __shared__ TileShared sh;
    __shared__ int64_t s_base[kServeMaxJobs];
    for (int t = threadIdx.x; t < n_jobs; t += kT) s_base[t] = jobs[t].tile_base;
    __syncthreads();
    const int64_t g = xcd_block(blockIdx.x, gridDim.x);
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_base[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    const JobDev J = jobs[lo];
    const int64_t tile = g - J.tile_base;
    if (J.mode == 0)
        process_tile<true, TW>(J.m, J.frags, J.n, J.vw, J.tiles_x, J.bias, J.maxd, apron, cap, J.vec_ok, J.out,
                               tile, sh, s_tex);
    else
        process_tile<false, TW>(J.m, J.frags, J.n, J.vw, J.tiles_x, J.bias, J.maxd, apron, cap, J.vec_ok, J.out,
                                tile, sh, s_tex);
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
    int64_t off = -1, bytes = 0;         // arena block
    void *d_out[rbsm::kMaxLights]{};     // per-light device results (in the arena)
    float *d_comp = nullptr;             // device composite (in the arena), or null
    Clock::time_point t_submit, t_done;
    hipEvent_t done = nullptr;           // results are in the host buffers
    int status = 0;                      // 0 pending, 1 done, < 0 failed
};

struct Slot {
    JobDev *d_jobs = nullptr, *h_jobs = nullptr;
    rbsm::CompJob *d_comp = nullptr, *h_comp = nullptr;
    hipEvent_t compute_done = nullptr;
    bool busy = false;
};

int64_t request_bytes(const rbsm_request &r) {
    int64_t b = 0;
    for (int l = 0; l < r.n_lights; ++l) b += rbsm::Arena::round_up(r.n * (r.lights[l].mode == 0 ? 1 : 4));
    if (r.composite_host) b += rbsm::Arena::round_up(r.n * 4);
    return b;
}

}  // namespace

struct rbsm_engine {
    int device = 0;
    char *d_arena = nullptr;
    rbsm::Arena arena;  // worker thread only
    int32_t max_inflight = 1;
    hipStream_t s_compute = nullptr, s_copy = nullptr;
    Slot slots[rbsm::kServeSlots];
    std::vector<std::vector<EngineReq *>> slot_reqs = std::vector<std::vector<EngineReq *>>(rbsm::kServeSlots);

    std::mutex mu;  // guards everything below
    std::condition_variable cv_work, cv_done;
    std::vector<MapView> lights;
    std::deque<EngineReq *> queue;                   // submitted, not admitted
    std::unordered_map<int64_t, EngineReq *> tickets;  // not yet collected by wait()
    int64_t next_ticket = 1;
    bool stop = false;
    std::string error;
    rbsm_engine_stats stats{};

    std::vector<EngineReq *> admitted;  // worker thread only
    std::vector<EngineReq *> inflight;  // worker thread only
    std::thread worker;

    void run();
    bool step_launch();
    void fail_all(const char *what, hipError_t e);
};

namespace {

// Build one scheduling step's tables for the admitted requests and enqueue
// it.  Returns false when nothing could be launched (no free slot).
int pick_slot(rbsm_engine *E) {
    int pending = 0, free_slot = -1;
    for (int s = 0; s < rbsm::kServeSlots; ++s) {
        if (E->slots[s].busy) ++pending;
        else if (free_slot < 0) free_slot = s;
    }
    return pending < rbsm::kServeComputeAhead ? free_slot : -1;
}

}  // namespace

void rbsm_engine::fail_all(const char *what, hipError_t e) {
    std::lock_guard<std::mutex> lk(mu);
    if (error.empty()) error = std::string(what) + ": " + hipGetErrorString(e);
    for (auto *r : admitted) r->status = RBSM_ERR_HIP;
    for (auto *r : inflight) r->status = RBSM_ERR_HIP;
    for (auto *r : queue) r->status = RBSM_ERR_HIP;
    admitted.clear();
    inflight.clear();
    queue.clear();
    cv_done.notify_all();
}

bool rbsm_engine::step_launch() {
    const int s = pick_slot(this);
    if (s < 0 || admitted.empty()) return false;
    Slot &S = slots[s];
    std::vector<EngineReq *> batch;
    std::vector<std::pair<EngineReq *, int>> rpcf_jobs;
    int n_jobs = 0, n_comp = 0;
    int64_t tiles = 0, comp_blocks = 0;
    size_t taken = 0;
    for (; taken < admitted.size(); ++taken) {
        EngineReq *R = admitted[taken];
        const rbsm_request &q = R->req;
        int tile_jobs = 0;
        for (int l = 0; l < q.n_lights; ++l) tile_jobs += (q.lights[l].kernel_radius == 0);
        if (n_jobs + tile_jobs > rbsm::kServeMaxJobs || (int)batch.size() >= rbsm::kServeMaxReqs) break;
        for (int l = 0; l < q.n_lights; ++l) {
            const rbsm_request_light &L = q.lights[l];
            if (L.kernel_radius > 0) {
                rpcf_jobs.push_back({R, l});
                continue;
            }
            const JobLayout lay = job_layout(q.n, q.view_width, kDefaultTile.tile_w);
            JobDev &D = S.h_jobs[n_jobs++];
            D.m = R->maps[l];
            D.frags = L.frags;
            D.out = R->d_out[l];
            D.n = q.n;
            D.vw = lay.vw;
            D.tiles_x = lay.tiles_x;
            D.tile_base = tiles;
            D.bias = L.depth_bias;
            D.maxd = L.max_dist;
            D.mode = L.mode;
            D.vec_ok = ((uintptr_t)L.frags % 16 == 0) && (lay.vw % 4 == 0);  // arena outputs are 256-aligned
            tiles += lay.tiles;
        }
        if (R->d_comp) {
            rbsm::CompJob &C = S.h_comp[n_comp++];
            C.n_lights = q.n_lights;
            C.n = q.n;
            C.out = R->d_comp;
            C.block_base = comp_blocks;
            for (int l = 0; l < q.n_lights; ++l) {
                C.vis[l] = R->d_out[l];
                C.w[l] = q.lights[l].weight;
                C.hard[l] = q.lights[l].mode == 0;
            }
            comp_blocks += rbsm::composite_blocks(q.n);
        }
        batch.push_back(R);
    }
    if (batch.empty()) return false;
    admitted.erase(admitted.begin(), admitted.begin() + taken);

    hipError_t e = hipSuccess;
    if (n_jobs > 0)
        e = hipMemcpyAsync(S.d_jobs, S.h_jobs, sizeof(JobDev) * n_jobs, hipMemcpyHostToDevice, s_compute);
    if (e == hipSuccess && n_comp > 0)
        e = hipMemcpyAsync(S.d_comp, S.h_comp, sizeof(rbsm::CompJob) * n_comp, hipMemcpyHostToDevice, s_compute);
    if (e != hipSuccess) {
        fail_all("engine: table upload", e);
        return false;
    }
    if (tiles > 0) {
        const size_t lds = (size_t)kDefaultTile.cap * sizeof(float);
        hipLaunchKernelGGL(rbsm::serve_kernel<32>, dim3((unsigned)tiles), dim3(kT), lds, s_compute, S.d_jobs, n_jobs,
                           kDefaultTile.apron, kDefaultTile.cap);
    }
    for (const auto &rj : rpcf_jobs) {
        const rbsm_request &q = rj.first->req;
        const rbsm_request_light &L = q.lights[rj.second];
        launch_rpcf(rj.first->maps[rj.second], L.frags, q.n, q.view_width, L.depth_bias, L.max_dist, L.kernel_radius,
                    static_cast<float *>(rj.first->d_out[rj.second]), s_compute);
    }
    if (comp_blocks > 0)
        hipLaunchKernelGGL(rbsm::composite_batch_kernel, dim3((unsigned)comp_blocks), dim3(rbsm::kCompT), 0, s_compute,
                           S.d_comp, n_comp);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(S.compute_done, s_compute);
    if (e == hipSuccess) e = hipStreamWaitEvent(s_copy, S.compute_done, 0);
    for (EngineReq *R : batch) {
        const rbsm_request &q = R->req;
        for (int l = 0; l < q.n_lights && e == hipSuccess; ++l)
            if (q.lights[l].out_host && q.n > 0)
                e = hipMemcpyAsync(q.lights[l].out_host, R->d_out[l], (size_t)q.n * (q.lights[l].mode == 0 ? 1 : 4),
                                   hipMemcpyDeviceToHost, s_copy);
        if (e == hipSuccess && R->d_comp && q.n > 0)
            e = hipMemcpyAsync(q.composite_host, R->d_comp, (size_t)q.n * 4, hipMemcpyDeviceToHost, s_copy);
        if (e == hipSuccess) e = hipEventRecord(R->done, s_copy);
        inflight.push_back(R);
    }
    if (e != hipSuccess) {
        fail_all("engine: launch", e);
        return false;
    }
    S.busy = true;
    slot_reqs[s] = batch;
    {
        std::lock_guard<std::mutex> lk(mu);
        stats.launches += 1;
        stats.jobs_launched += n_jobs + (int64_t)rpcf_jobs.size();
    }
    return true;
}

void rbsm_engine::run() {
    (void)hipSetDevice(device);
    for (;;) {
        bool progress = false;
        // steps whose compute finished free their table slot
        for (int s = 0; s < rbsm::kServeSlots; ++s) {
            if (!slots[s].busy) continue;
            const hipError_t q = hipEventQuery(slots[s].compute_done);
            if (q == hipSuccess) {
                slots[s].busy = false;
                slot_reqs[s].clear();
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
            arena.release(R->off, R->bytes);
            std::lock_guard<std::mutex> lk(mu);
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
                const int64_t off = arena.alloc(R->bytes);
                if (off < 0) break;
                R->off = off;
                char *p = d_arena + off;
                for (int l = 0; l < R->req.n_lights; ++l) {
                    R->d_out[l] = p;
                    p += rbsm::Arena::round_up(R->req.n * (R->req.lights[l].mode == 0 ? 1 : 4));
                }
                R->d_comp = R->req.composite_host ? reinterpret_cast<float *>(p) : nullptr;
                queue.pop_front();
                admitted.push_back(R);
                stats.queued -= 1;
                stats.inflight += 1;
                stats.arena_peak_bytes = arena.peak();
                progress = true;
            }
        }
        if (step_launch()) progress = true;
        if (!progress) {
            std::unique_lock<std::mutex> lk(mu);
            if (stop && queue.empty() && admitted.empty() && inflight.empty()) break;
            if (queue.empty() && admitted.empty() && inflight.empty())
                cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            else
                cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}
