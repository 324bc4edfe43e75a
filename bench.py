"""Benchmark of the RBSM per-fragment shadow pass on one MI355X.

One step = one frame of the batched workload through the whole hot path:
16 shadow maps of uneven sizes (a directional light's cascades 8192^2 ..
1024^2 and 12 spot maps 1024^2 .. 4096^2, random-triangle scenes) and 8 views
(two each of 1280x720, 1920x1080, 2560x1440, 3840x2160) split into 48
(view, light) jobs -- hard RBSM on the cascades, RSMSS radius 0 on the spot
lights -- 66.55 M fragment evaluations, run as one replay of the captured
batched plan.  The frame's inputs (1.6 GB) are resident in HBM before timing
and exceed the 256 MB last-level cache, so every frame streams from HBM.

Prints ONE JSON line: the headline (batched fragments/s), the plain
per-view launches of the same jobs, p50/p99 frame latency, the dominant
kernel's roofline (algorithmic bytes / kernel time from HIP events on its
launch stream), extras (the single-view hard pass at 2048^2 / 1080p, RSMSS
and RPCF at 4K, 512^2 uniform frames, the per-light-radius batched variant,
serving, rasterization, compositing) and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shaded fragments/sec (RBSM, RSMSS) batched vs plain per-view; p99 frame latency"
PEAK_HBM_GBPS = 8000.0
ROTATE_BYTES = 512 << 20
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "batch_arg_kernel_16maps_8views_traffic.md")


def code_tokens(text: str) -> str:
    """C++ source without its comments and with runs of white space made one
    space: what the compiler sees, so edits of comments keep the hash."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    """Hash of the code (comments aside) that defines the tile-pass kernels:
    the tile pass and the per-fragment device helpers."""
    h = hashlib.sha256()
    for rel in ("paper_1711_07793_amd/csrc/tile_pass.hpp", "paper_1711_07793_amd/csrc/rbsm_device.hpp"):
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


def read_traffic(kernel_hash: str, tuning: dict, path: str = PROFILE_TRAFFIC):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing, was taken on a different kernel source, or holds
    no entry for this launch tuning.  The summary ends with lines
    ``- kernel_source_sha: `<sha>` `` and, per profiled tuning,
    ``- hbm_bytes_per_launch <tuning label>: `<bytes>` ``."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha") != kernel_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch " + tuning_label(tuning)])
    except (KeyError, ValueError):
        return None


def tuning_label(t: dict) -> str:
    return ",".join(f"{k}={t[k]}" for k in ("tile_w", "apron", "lds_cap", "persistent", "walk_first", "walk_block",
                                            "xcd_chunk"))


ARG_JOBS_MAX = 48  # jobs with tiles whose records a one-shot launch takes in its kernel arguments


def kernel_instance(t: dict, tiled_jobs: int) -> str:
    """Name of the batched kernel a tuning launches for a plan with
    `tiled_jobs` jobs in the tile pass."""
    if t["persistent"]:
        return f"batch_persistent_kernel<{t['tile_w']}, {t['walk_first']}, {t['walk_block']}>"
    name = "batch_arg_kernel" if tiled_jobs <= ARG_JOBS_MAX else "batch_kernel"
    return f"{name}<{t['tile_w']}, {t['walk_first']}, {t['walk_block']}>"


class Frames:
    """Distinct device copies of a few generated frames, rotated per step."""

    def __init__(self, torch, cfg: int, seeds, min_bytes: int, mode: str, out_dtype):
        import synth
        self.inputs = []
        host = [synth.make_config(cfg, s) for s in seeds]
        self.host = host
        per = host[0]["map"].nbytes + host[0]["frags"].nbytes
        n_copies = max(len(host), -(-min_bytes // per))
        self.slots = []
        for k in range(n_copies):
            h = host[k % len(host)]
            m = torch.from_numpy(h["map"]).cuda()
            f = torch.from_numpy(h["frags"]).cuda()
            o = torch.empty(len(h["frags"]), dtype=out_dtype, device="cuda")
            self.slots.append((k % len(host), m, f, o))
        self.n = len(host[0]["frags"])
        self.params = host[0]["params"]
        self.bytes_resident = n_copies * (per + self.slots[0][3].numel() * self.slots[0][3].element_size())


def time_pass(torch, rb, lib, fn_name, frames: Frames, params, steps: int, warmup: int):
    """Warm up, then time exactly `steps` back-to-back launches, synchronised on
    both sides.  One HIP event pair on the launch stream brackets the timed
    region, so the average launch duration is the event time over `steps`
    (kernel time plus the back-to-back dispatch gap, nothing from the host).
    Returns (wall seconds, average launch ms, slot index of every step)."""
    p = rb.Params(**params).to_c()
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    fn = getattr(lib, fn_name)
    args = [(s[1].data_ptr(), s[2].data_ptr(), frames.n, ctypes.byref(p), s[3].data_ptr()) for s in frames.slots]
    nslot = len(args)
    for k in range(warmup):
        a = args[k % nslot]
        st = fn(a[0], a[1], a[2], a[3], a[4], sh)
        assert st == 0, rb.rbsm_last_error()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    # the timed steps continue the rotation, so the first of them reads the
    # slot touched longest ago, not one the warm-up left in the cache
    first = warmup % nslot
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(steps):
        a = args[(first + k) % nslot]
        fn(a[0], a[1], a[2], a[3], a[4], sh)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_ms = ev0.elapsed_time(ev1) / steps
    used = [(first + k) % nslot for k in range(steps)]
    return wall, avg_ms, used


def launch_latency(torch, rb, lib, fn_name, frames: Frames, params, count: int):
    """Per-frame latency: `count` single launches, each bracketed by its own
    event pair and synchronised before the next (dispatch included)."""
    p = rb.Params(**params).to_c()
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    fn = getattr(lib, fn_name)
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lat = []
    for k in range(count):
        sl = frames.slots[k % len(frames.slots)]
        s0.record(stream)
        fn(sl[1].data_ptr(), sl[2].data_ptr(), frames.n, ctypes.byref(p), sl[3].data_ptr(), sh)
        s1.record(stream)
        s1.synchronize()
        lat.append(s0.elapsed_time(s1))
    lat = np.array(lat)
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def algorithmic_bytes(torch, rb, frames: Frames, params, mode: int, out_bytes: int):
    """Per-frame algorithmic bytes: 12 B per fragment in, the output, and
    4 B per distinct texel the pass reads (counted on the device)."""
    per_frame = []
    for h in frames.host:
        m = torch.from_numpy(h["map"]).cuda()
        f = torch.from_numpy(h["frags"]).cuda()
        t = rb.rbsm_footprint(m, f, params, mode)
        texels = int(t.sum().item())
        per_frame.append(12 * frames.n + out_bytes * frames.n + 4 * texels)
    return per_frame


def copy_bandwidth(torch, nbytes: int = 256 << 20, reps: int = 5) -> float:
    """Read + write bandwidth of a plain device-to-device copy of nbytes."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        dst.copy_(src)
    e.record()
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (s.elapsed_time(e) * 1e-3) / 1e9


class BatchedFrame:
    """The batched workload on the device: 16 maps, 8 views, 48 jobs (one
    output buffer per job), plus the frame's algorithmic bytes."""

    def __init__(self, torch, rb, seed: int = 4001, radius_per_light: bool = False):
        import synth
        w = synth.make_batched(seed)
        self.maps = [torch.from_numpy(m).cuda() for m in w["maps"]]
        self.jobs = []
        radii = {}
        for j in w["jobs"]:
            params = dict(j["params"])
            if radius_per_light and j["mode"] == 1:
                # each spot light's own kernel radius 3..15 (one per light)
                radii.setdefault(j["map"], 3 + int(synth.uniform_floats(seed * 7 + j["map"], 1)[0] * 13))
                params["kernel_radius"] = radii[j["map"]]
            f = torch.from_numpy(j["frags"]).cuda()
            out = torch.empty(len(j["frags"]), dtype=torch.uint8 if j["mode"] == 0 else torch.float32, device="cuda")
            self.jobs.append(dict(map=self.maps[j["map"]], frags=f, params=params, mode=j["mode"], out=out))
        self.radii = radii
        self.n_frag = sum(j["frags"].numel() // 3 for j in self.jobs)
        # jobs in the tile pass (RPCF jobs run their own kernel)
        self.tiled_jobs = sum(1 for j in self.jobs if j["frags"].numel() > 0 and
                              not (j["mode"] == 1 and j["params"].get("kernel_radius", 0) > 0))
        self.resident_bytes = sum(t.numel() * t.element_size() for t in self.maps) + sum(
            j["frags"].numel() * 4 + j["out"].numel() * j["out"].element_size() for j in self.jobs)
        lib = rb.load_library()
        self.cparams = [rb.Params(**j["params"]).to_c() for j in self.jobs]
        self.lib = lib

    def frame_bytes(self, rb) -> int:
        """12 B per fragment in, 1 (hard) or 4 (RSMSS) B out, and 4 B per
        distinct texel each job reads (counted on the device)."""
        total = 0
        for j in self.jobs:
            n = j["frags"].numel() // 3
            t = rb.rbsm_footprint(j["map"], j["frags"], j["params"], j["mode"])
            total += (12 + (1 if j["mode"] == 0 else 4)) * n + 4 * int(t.sum().item())
            del t
        return total

    def plain_frame(self, stream_handle: int):
        """One call per job (the plain entry points), in job order."""
        for j, p in zip(self.jobs, self.cparams):
            fn = self.lib.rbsm_visibility if j["mode"] == 0 else self.lib.rsmss_visibility
            st = fn(j["map"].data_ptr(), j["frags"].data_ptr(), j["frags"].numel() // 3, ctypes.byref(p),
                    j["out"].data_ptr(), stream_handle)
            assert st == 0, self.lib.rbsm_last_error()

    def outputs(self):
        return [j["out"].clone() for j in self.jobs]

    def equal(self, want) -> bool:
        import torch
        return all(torch.equal(j["out"], w) for j, w in zip(self.jobs, want))


def frame_rate(torch, frame_fn, sync_fn, n_frag: int, frames: int, warmup: int = 3):
    """Frames run one at a time, each synchronised (a renderer waiting for
    its shadow buffers): fragments/s and p50/p99 frame latency (host clock)."""
    for _ in range(warmup):
        frame_fn()
    sync_fn()
    lat = []
    t0 = time.perf_counter()
    for _ in range(frames):
        a = time.perf_counter()
        frame_fn()
        sync_fn()
        lat.append((time.perf_counter() - a) * 1e3)
    wall = time.perf_counter() - t0
    lat = np.array(lat)
    return {"fragments_per_s": n_frag * frames / wall, "p50_frame_ms": float(np.percentile(lat, 50)),
            "p99_frame_ms": float(np.percentile(lat, 99)), "frames": frames}


def batched_headline(torch, rb, bf: BatchedFrame, steps: int, warmup: int, latency_frames: int = 200,
                     fixed_tuning=None):
    """The headline: plain per-view launches of the 48 jobs, then the
    autotuned (or, with fixed_tuning, the given) batched plan captured as a
    HIP graph.  Exactly `steps` graph replays run back to back between
    synchronisations; one HIP event pair on the replay stream brackets them
    (the kernel's average duration)."""
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    plain = frame_rate(torch, lambda: bf.plain_frame(sh), torch.cuda.synchronize, bf.n_frag, 30)
    want = bf.outputs()
    plan = rb.Plan(bf.jobs)
    if fixed_tuning is None:
        tune = plan.autotune(reps=10).as_dict()
    else:
        plan.tuning = fixed_tuning
        tune = plan.tuning.as_dict()
    for j in bf.jobs:
        j["out"].fill_(0)
    plan.launch()
    torch.cuda.synchronize()
    equal = bf.equal(want)
    eager = frame_rate(torch, plan.launch, torch.cuda.synchronize, bf.n_frag, 30)
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    plan.capture(s)
    for _ in range(warmup):
        plan.launch(s)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(s)
    for _ in range(steps):
        plan.launch(s)
    ev1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_ms = ev0.elapsed_time(ev1) / steps
    graph_equal = bf.equal(want)
    # per-frame latency: single replays, each bracketed by events and waited for
    lat = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(latency_frames):
        e0.record(s)
        plan.launch(s)
        e1.record(s)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    lat = np.array(lat)
    plan.close()
    return {
        "wall_s": wall, "avg_kernel_ms": avg_ms, "tuning": tune,
        "p50_frame_ms": float(np.percentile(lat, 50)), "p99_frame_ms": float(np.percentile(lat, 99)),
        "plain_per_view": plain, "batched_eager": eager,
        "bitwise_equal_to_plain": bool(equal and graph_equal),
    }


def batched_radius_section(torch, rb, frames: int = 10):
    """The per-light-radius variant of the batched workload: every spot light
    filters with its own RPCF radius 3..15 (RSMSS box-averaged), cascades stay
    hard.  Plain per-view launches vs the plan (one graph replay per frame)."""
    bf = BatchedFrame(torch, rb, radius_per_light=True)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    plain = frame_rate(torch, lambda: bf.plain_frame(sh), torch.cuda.synchronize, bf.n_frag, frames, warmup=1)
    want = bf.outputs()
    plan = rb.Plan(bf.jobs)
    plan.autotune(reps=1)
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    plan.capture(s)
    for j in bf.jobs:
        j["out"].fill_(0)
    graph = frame_rate(torch, lambda: plan.launch(s), s.synchronize, bf.n_frag, frames, warmup=1)
    equal = bf.equal(want)
    plan.close()
    terms = sum((j["frags"].numel() // 3) * (2 * j["params"]["kernel_radius"] + 1) ** 2 for j in bf.jobs)
    return {"workload": "batched workload with each spot light's own RPCF radius "
                        f"({sorted(set(bf.radii.values()))}), cascades hard",
            "fragments_per_frame": bf.n_frag, "rsmss_terms_per_frame": terms,
            "plain_per_view": plain, "batched_graph": graph,
            "speedup_vs_plain": graph["fragments_per_s"] / plain["fragments_per_s"],
            "bitwise_equal_to_plain": bool(equal)}


def serving_section(torch, rb, n_requests: int = 10000, seed: int = 5001, budget: int = 4 << 30,
                    concurrency: int = 32, loads=(0.25, 0.5, 0.75, 0.9),
                    budgets=(768 << 20, 1 << 30, 2 << 30, 4 << 30, 8 << 30)):
    """Serving workload: a pool of 16 resident lights (random-triangle maps,
    four each of 1024^2, 2048^2, 4096^2 and 8192^2, rasterized on the device),
    views of 1280x720 / 1920x1080 / 3840x2160 whose light-space fragments are
    device-resident, and n_requests requests of 1-4 distinct lights, each
    light hard or RSMSS r=0 with equal odds, equal weights; the result is the
    view's composite shadow buffer in device memory.  Compared: plain
    per-request launches (one call per light, compositing, synchronise) vs
    the engine (continuous batching under an HBM budget on the working sets
    of admitted requests): saturation throughput with `concurrency` requests
    outstanding, then p50/p99 latency under Poisson arrivals at fractions of
    the plain path's saturation rate, then engine saturation across budgets."""
    import threading
    import synth
    lib = rb.load_library()
    rng = np.random.default_rng(seed)
    sizes = [1024, 2048, 4096, 8192] * 4
    views = [(1280, 720), (1920, 1080), (3840, 2160)]
    maps, frags = [], {}
    for li, S in enumerate(sizes):
        sc = synth.triangle_scene(seed * 10 + li, S, S, 64)
        prims, rec = sc.primitives()
        dp = torch.from_numpy(np.ascontiguousarray(prims).view(np.uint8).copy()).cuda()
        m = torch.empty((S, S), dtype=torch.float32, device="cuda")
        rb.rbsm_rasterize(dp, rec, S, S, out=m)
        maps.append(m)
        for vi, (w, h) in enumerate(views):
            frags[(li, vi)] = torch.from_numpy(sc.camera_fragments(seed * 100 + 10 * li + vi, w, h)).cuda()
    torch.cuda.synchronize()
    reqs = []
    for _ in range(n_requests):
        vi = int(rng.integers(0, 3))
        nl = int(rng.integers(1, 5))
        ls = [int(x) for x in rng.choice(16, size=nl, replace=False)]
        modes = [int(x) for x in rng.integers(0, 2, size=nl)]
        reqs.append((vi, ls, modes))
    evals = np.array([views[vi][0] * views[vi][1] * len(ls) for vi, ls, _ in reqs], dtype=np.float64)
    ring = concurrency + 16
    dest = {vi: [torch.empty(w * h, dtype=torch.float32, device="cuda") for _ in range(ring)]
            for vi, (w, h) in enumerate(views)}
    nmax = views[2][0] * views[2][1]
    dev_out = [torch.empty(nmax * 4, dtype=torch.uint8, device="cuda") for _ in range(4)]
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    cparams = {(li, vi): rb.Params(width=sizes[li], height=sizes[li], depth_bias=1e-4, max_dist=16,
                                   view_width=views[vi][0]).to_c() for li in range(16) for vi in range(3)}

    def plain(q, slot):
        vi, ls, modes = reqs[q]
        n = views[vi][0] * views[vi][1]
        ptrs = []
        for k, (li, mode) in enumerate(zip(ls, modes)):
            fn = lib.rbsm_visibility if mode == 0 else lib.rsmss_visibility
            st = fn(maps[li].data_ptr(), frags[(li, vi)].data_ptr(), n, ctypes.byref(cparams[(li, vi)]),
                    dev_out[k].data_ptr(), sh)
            assert st == 0, rb.rbsm_last_error()
            ptrs.append(dev_out[k].data_ptr())
        L = len(ls)
        out = dest[vi][slot % ring]
        st = lib.rbsm_composite(n, L, (ctypes.c_void_p * L)(*ptrs), (ctypes.c_int32 * L)(*modes),
                                (ctypes.c_float * L)(*([1.0 / L] * L)), out.data_ptr(), sh)
        assert st == 0, rb.rbsm_last_error()
        stream.synchronize()
        return out

    def make_engine(b):
        eng = rb.Engine(b, concurrency)
        return eng, [eng.add_light(m) for m in maps]

    def build(eng, ids, q, slot):
        vi, ls, modes = reqs[q]
        n = views[vi][0] * views[vi][1]
        L = [dict(light=ids[li], mode=mode, frags=frags[(li, vi)], depth_bias=1e-4, max_dist=16,
                  weight=1.0 / len(ls)) for li, mode in zip(ls, modes)]
        return eng.build_request(n, L, view_width=views[vi][0], composite=dest[vi][slot % ring])[0]

    tk = ctypes.c_int64()

    def submit(eng, req):
        st = lib.rbsm_engine_submit(eng._h, ctypes.byref(req), ctypes.byref(tk))
        assert st == 0, rb.rbsm_last_error()
        return int(tk.value)

    eng, ids = make_engine(budget)
    built = [build(eng, ids, q, q) for q in range(n_requests)]  # marshalled ahead, as a native front end would

    # identical accuracy: the engine's composites equal the plain path's bitwise
    equal = True
    for q in range(16):
        want = plain(q, 0).clone()
        t = submit(eng, build(eng, ids, q, 1))
        eng.wait(t)
        equal &= bool(torch.equal(dest[reqs[q][0]][1], want))

    for q in range(32):  # warm-up
        plain(q, q)
        eng.wait(submit(eng, built[q]))

    def engine_saturation(e, b_reqs):
        busy0 = e.stats()["gpu_busy_ns"]
        t0 = time.perf_counter()
        pending = []
        for q in range(n_requests):
            if len(pending) >= concurrency:
                lib.rbsm_engine_wait(e._h, pending.pop(0), -1, None)
            pending.append(submit(e, b_reqs[q]))
        for t in pending:
            lib.rbsm_engine_wait(e._h, t, -1, None)
        dt = time.perf_counter() - t0
        return dt, (e.stats()["gpu_busy_ns"] - busy0) * 1e-9

    t0 = time.perf_counter()
    for q in range(n_requests):
        plain(q, q)
    plain_s = time.perf_counter() - t0
    serve_s, busy_s = engine_saturation(eng, built)
    plain_rate = n_requests / plain_s
    total_evals = float(evals.sum())

    def poisson(frac):
        lam = frac * plain_rate
        arr = np.cumsum(rng.exponential(1.0 / lam, size=n_requests))
        lat_p = []
        t0 = time.perf_counter()
        for q in range(n_requests):
            now = time.perf_counter() - t0
            if now < arr[q]:
                time.sleep(arr[q] - now)
            plain(q, q)
            lat_p.append((time.perf_counter() - t0 - arr[q]) * 1e3)
        tickets = [None] * n_requests

        def producer():
            t1 = time.perf_counter()
            for q in range(n_requests):
                now = time.perf_counter() - t1
                if now < arr[q]:
                    time.sleep(arr[q] - now)
                tickets[q] = submit(eng, built[q])

        lat_s = []
        th = threading.Thread(target=producer)
        th.start()
        for q in range(n_requests):
            while tickets[q] is None:
                time.sleep(5e-5)
            lat_s.append(eng.wait(tickets[q]))
        th.join()
        pct = lambda a, p: float(np.percentile(np.array(a), p))
        return {"offered_req_per_s": lam,
                "plain": {"p50_ms": pct(lat_p, 50), "p99_ms": pct(lat_p, 99)},
                "engine": {"p50_ms": pct(lat_s, 50), "p99_ms": pct(lat_s, 99)}}

    pois = {f"{f}x_plain_saturation": poisson(f) for f in loads}
    st = eng.stats()
    eng.close()
    sweep = {}
    for b in budgets:
        e2, ids2 = make_engine(b)
        b_reqs = [build(e2, ids2, q, q) for q in range(n_requests)]
        for q in range(8):
            e2.wait(submit(e2, b_reqs[q]))
        dt, _ = engine_saturation(e2, b_reqs)
        s2 = e2.stats()
        sweep[str(b)] = {"requests_per_s": n_requests / dt, "fragments_per_s": total_evals / dt,
                         "inflight_peak_bytes": s2["inflight_peak_bytes"], "launches": s2["launches"]}
        e2.close()
    return {
        "workload": "16 resident lights (4 each of 1024^2, 2048^2, 4096^2, 8192^2 maps of 64 triangles, rasterized "
                    "on the device), views 720p/1080p/4K with device-resident light-space fragments, "
                    f"{n_requests} requests of 1-4 lights (each hard or RSMSS r=0), composite to a device buffer",
        "requests": n_requests,
        "fragment_evaluations": total_evals,
        "hbm_budget_bytes": budget,
        "plain_saturation": {"requests_per_s": plain_rate, "fragments_per_s": total_evals / plain_s},
        "engine_saturation": {"requests_per_s": n_requests / serve_s, "fragments_per_s": total_evals / serve_s,
                              "outstanding": concurrency, "gpu_busy_fraction": busy_s / serve_s},
        "speedup_vs_plain": plain_s / serve_s,
        "poisson": pois,
        "budget_sweep": sweep,
        "engine_stats": {"launches": st["launches"], "jobs_launched": st["jobs_launched"],
                         "inflight_peak_bytes": st["inflight_peak_bytes"]},
        "bitwise_equal_to_plain": equal,
    }


def raster_section(torch, rb, seed: int = 5001, reps: int = 10):
    """On-device shadow-map rasterization of the serving lights' scenes
    (64-triangle scenes, 1024^2..8192^2): time per map and texel rate; the
    pass writes 4 bytes per texel."""
    import synth
    res = {}
    for S in (1024, 2048, 4096, 8192):
        sc = synth.triangle_scene(seed * 10 + {1024: 0, 2048: 1, 4096: 2, 8192: 3}[S], S, S, 64)
        prims, rec = sc.primitives()
        dp = torch.from_numpy(np.ascontiguousarray(prims).view(np.uint8).copy()).cuda()
        out = torch.empty((S, S), dtype=torch.float32, device="cuda")
        rb.rbsm_rasterize(dp, rec, S, S, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            rb.rbsm_rasterize(dp, rec, S, S, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[f"{S}x{S}"] = {"ms": ms, "texels_per_s": S * S / (ms * 1e-3), "write_GBps": 4 * S * S / (ms * 1e-3) / 1e9}
    return {"workload": "64 random triangles over a tilted receiver, binary64 coverage", "maps": res}


def composite_section(torch, rb, reps: int = 50):
    """Multi-light compositing of one 4K view: 2 hard masks and 2 RSMSS
    visibilities (1 + 1 + 4 + 4 bytes per fragment in) into a float32 shadow
    buffer (4 bytes out); time per launch and bandwidth against HBM."""
    n = 3840 * 2160
    g = torch.Generator(device="cuda").manual_seed(9)
    vis = [(torch.rand(n, device="cuda", generator=g) < 0.5).to(torch.uint8) for _ in range(2)]
    vis += [torch.rand(n, device="cuda", generator=g) for _ in range(2)]
    modes, weights = [0, 0, 1, 1], [0.4, 0.3, 0.2, 0.1]
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    rb.rbsm_composite(vis, modes, weights, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rb.rbsm_composite(vis, modes, weights, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = n * (1 + 1 + 4 + 4 + 4)
    return {"workload": "4 lights (2 hard, 2 RSMSS) composited over one 3840x2160 view", "ms": ms,
            "bytes_per_launch": nbytes, "achieved_GBps": nbytes / (ms * 1e-3) / 1e9, "hbm_peak_GBps": 8000.0}


def host_threads() -> tuple:
    """Threads for the CPU leg: the CPUs this process may run on (its
    affinity), capped by OMP_NUM_THREADS where the host sets one (a GPU machine
    gives each GPU a share of its cores that way).  Returns (threads,
    affinity size, os.cpu_count())."""
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = min(aff, cap) if cap > 0 else aff
    return max(1, threads), aff, os.cpu_count()


def cpu_baseline(budget_s: float, subset: int = 1 << 20, seed: int = 4001):
    """The oracle (single-threaded C, unchanged) on a fixed 2^20-fragment
    subset of the batched workload: every job contributes the same share of
    its rows, so the subset keeps the frame's mix of maps, modes and views.
    Passes over the subset repeat for budget_s / 2 on one thread, then for
    budget_s / 2 fanned out over the host's threads by static fragment
    slices (the C calls release the interpreter lock).  Reported value: the
    all-threads rate."""
    import threading
    import oracle
    import synth
    w = synth.make_batched(seed)
    total = sum(len(j["frags"]) for j in w["jobs"])
    parts = []
    for j in w["jobs"]:
        k = max(1, round(len(j["frags"]) * subset / total))
        parts.append((w["maps"][j["map"]], np.ascontiguousarray(j["frags"][:k]), j["params"], j["mode"]))
    n_sub = sum(len(p[1]) for p in parts)

    def run_slice(a, b):
        """Fragments [a, b) of the subset (in job order)."""
        done, base = 0, 0
        for m, f, prm, mode in parts:
            lo, hi = max(a - base, 0), min(b - base, len(f))
            if lo < hi:
                (oracle.rbsm_hard if mode == 0 else oracle.rsmss)(m, f[lo:hi], prm)
                done += hi - lo
            base += len(f)
        return done

    def run_for(seconds, threads):
        done = [0] * threads
        stop = time.perf_counter() + seconds

        def worker(t):
            a, b = n_sub * t // threads, n_sub * (t + 1) // threads
            while True:
                done[t] += run_slice(a, b)
                if time.perf_counter() >= stop:
                    break

        t0 = time.perf_counter()
        ts = [threading.Thread(target=worker, args=(t,)) for t in range(threads)]
        for th in ts:
            th.start()
        for th in ts:
            th.join()
        dt = time.perf_counter() - t0
        return sum(done) / dt, sum(done), dt

    single, n1, dt1 = run_for(budget_s / 2, 1)
    threads, aff, ncpu = host_threads()
    multi, nm, dtm = run_for(budget_s / 2, threads)
    return dict(value=multi, unit="fragments/s", cores=threads, kind="oracle",
                single_thread_value=single, host_cpu_count=ncpu, affinity_cpus=aff,
                omp_num_threads=os.environ.get("OMP_NUM_THREADS"),
                sample=f"fixed {n_sub}-fragment subset of the batched workload (every job's first rows, in "
                       f"proportion): {n1} fragments in {dt1:.1f} s on one thread, then {nm} fragments in "
                       f"{dtm:.1f} s on {threads} threads (static slices)")


def uniform_section(torch, rb, steps: int = 2000, n_frames: int = 280):
    """The 512^2 single-quad workload: 65,536 uniformly scattered fragments per
    frame (no screen locality), hard RBSM, MAXDIST 16.  n_frames distinct
    frames (>= 512 MB) rotate through the timed launches."""
    import synth
    lib = rb.load_library()
    slots = []
    for k in range(n_frames):
        c = synth.make_config(1, 1000 + 1 + k)
        m = torch.from_numpy(c["map"]).cuda()
        f = torch.from_numpy(c["frags"]).cuda()
        o = torch.empty(len(c["frags"]), dtype=torch.uint8, device="cuda")
        slots.append((m, f, o, rb.Params(**c["params"]).to_c()))
    n = len(c["frags"])
    resident = n_frames * (512 * 512 * 4 + n * 13)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    for k in range(20):
        m, f, o, p = slots[k % n_frames]
        assert lib.rbsm_visibility(m.data_ptr(), f.data_ptr(), n, ctypes.byref(p), o.data_ptr(), sh) == 0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(steps):
        m, f, o, p = slots[(20 + k) % n_frames]
        lib.rbsm_visibility(m.data_ptr(), f.data_ptr(), n, ctypes.byref(p), o.data_ptr(), sh)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_ms = ev0.elapsed_time(ev1) / steps
    # algorithmic bytes of a few frames: fragments in, mask out, distinct texels
    per = []
    for m, f, o, p in slots[:8]:
        params = dict(width=512, height=512, pitch=512, depth_bias=1e-4, max_dist=16)
        t = rb.rbsm_footprint(m, f, params, 0)
        per.append(13 * n + 4 * int(t.sum().item()))
    b = float(np.mean(per))
    return {"workload": "hard RBSM, 512x512 map of one rotated quad, 65,536 uniform fragments per frame, MAXDIST 16",
            "frames_rotated": n_frames, "resident_bytes": resident, "fragments_per_s": n * steps / wall,
            "avg_kernel_ms": avg_ms, "algorithmic_bytes_per_launch": b,
            "achieved_GBps": b / (avg_ms * 1e-3) / 1e9}


def single_view_section(torch, rb, steps: int):
    """The single-view hard pass: 2048^2 map of 64 triangles, 1920x1080
    perspective fragments, MAXDIST 32; 13 distinct frames rotate."""
    lib = rb.load_library()
    frames = Frames(torch, 2, [2001, 2002, 2003, 2004, 2005], ROTATE_BYTES, "hard", torch.uint8)
    params = frames.params
    wall, avg_ms, used = time_pass(torch, rb, lib, "rbsm_visibility", frames, params, steps, 20)
    per_frame = algorithmic_bytes(torch, rb, frames, params, 0, 1)
    scene = [s[0] for s in frames.slots]
    bpl = float(np.mean([per_frame[scene[u]] for u in used]))
    p50, p99 = launch_latency(torch, rb, lib, "rbsm_visibility", frames, params, 300)
    w_sm, a_sm, _ = time_pass(torch, rb, lib, "sm_visibility", frames, params, max(200, steps // 4), 20)
    return {"workload": "hard RBSM, 2048x2048 map of 64 random triangles over a tilted receiver, 1920x1080 "
                        "perspective fragments, MAXDIST 32, one plain launch per frame",
            "fragments_per_s": frames.n * steps / wall, "ms_per_step": wall * 1e3 / steps,
            "avg_kernel_ms": avg_ms, "algorithmic_bytes_per_launch": bpl,
            "achieved_GBps": bpl / (avg_ms * 1e-3) / 1e9, "p50_frame_ms": p50, "p99_frame_ms": p99,
            "frames_rotated": len(frames.slots),
            "plain_sm": {"fragments_per_s": frames.n * max(200, steps // 4) / w_sm, "avg_kernel_ms": a_sm}}


def rsmss_section(torch, rb, steps: int):
    """RSMSS radius 0 and RPCF at the light's radius on the 4K fenced scene."""
    lib = rb.load_library()
    fr3 = Frames(torch, 3, [3001, 3002, 3003], ROTATE_BYTES, "rsmss", torch.float32)
    p3 = dict(fr3.params, kernel_radius=0)
    w3, a3, used3 = time_pass(torch, rb, lib, "rsmss_visibility", fr3, p3, steps, 10)
    b3 = algorithmic_bytes(torch, rb, fr3, p3, 1, 4)
    sc3 = [s[0] for s in fr3.slots]
    bpl3 = float(np.mean([b3[sc3[u]] for u in used3]))
    out = {"rsmss": {
        "workload": "RSMSS r=0, 4096x4096 map of 256 triangles + thin-bar fence, 3840x2160 fragments, MAXDIST 16",
        "fragments_per_s": fr3.n * steps / w3, "ms_per_step": w3 * 1e3 / steps, "avg_kernel_ms": a3,
        "achieved_GBps": bpl3 / (a3 * 1e-3) / 1e9, "algorithmic_bytes_per_launch": bpl3}}
    r3 = fr3.host[0]["light_radius"]
    pr = dict(fr3.params, kernel_radius=r3)
    steps_r = max(10, steps // 20)
    wr, ar, _ = time_pass(torch, rb, lib, "rsmss_visibility", fr3, pr, steps_r, 3)
    out["rpcf"] = {
        "workload": f"RPCF radius {r3} ({(2 * r3 + 1) ** 2} RSMSS terms per fragment) on the RSMSS frames",
        "kernel_radius": r3, "fragments_per_s": fr3.n * steps_r / wr, "ms_per_step": wr * 1e3 / steps_r,
        "avg_kernel_ms": ar, "terms_per_s": fr3.n * (2 * r3 + 1) ** 2 / (ar * 1e-3)}
    # the range of light radii the workload draws from (3-15), same frames
    sweep = {}
    for r in (3, 8, 15):
        _, a_r, _ = time_pass(torch, rb, lib, "rsmss_visibility", fr3, dict(fr3.params, kernel_radius=r),
                              max(5, steps // 40), 2)
        sweep[str(r)] = {"avg_kernel_ms": a_r, "terms_per_s": fr3.n * (2 * r + 1) ** 2 / (a_r * 1e-3)}
    out["rpcf"]["by_radius"] = sweep
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--tuning", default=None,
                    help="headline: launch this tuning (tile_w,apron,lds_cap,persistent,walk_first,walk_block,"
                         "xcd_chunk) instead of autotuning (for counter runs of one launch configuration)")
    ap.add_argument("--section", choices=["single_view_hard", "rsmss", "uniform_512", "serving"],
                    help="run only this extra section (for profiling) and print it as one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(every fragment/light evaluation is independent; multi-GPU sharding is described "
              "in the design notes but not run).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1711_07793_amd as rb

    rb.load_library()
    torch.cuda.init()

    if args.section:
        out = {}
        if args.copy_calibration:
            out["copy_kernel_GBps"] = copy_bandwidth(torch)
        if args.section == "single_view_hard":
            out[args.section] = single_view_section(torch, rb, args.steps)
        elif args.section == "rsmss":
            out.update(rsmss_section(torch, rb, args.steps))
        elif args.section == "uniform_512":
            out[args.section] = uniform_section(torch, rb, args.steps)
        else:
            out[args.section] = serving_section(torch, rb)
        print(json.dumps(out), flush=True)
        return

    # ---- headline: the batched workload, one graph replay per step --------
    bf = BatchedFrame(torch, rb)
    fixed = tuple(int(x) for x in args.tuning.split(",")) if args.tuning else None
    h = batched_headline(torch, rb, bf, args.steps, args.warmup, fixed_tuning=fixed)
    frame_bytes = bf.frame_bytes(rb)
    value = bf.n_frag * args.steps / h["wall_s"]
    achieved = frame_bytes / (h["avg_kernel_ms"] * 1e-3) / 1e9
    khash = kernel_source_hash()
    tune = h["tuning"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "fragments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched: 16 maps (cascades 8192^2, 4096^2, 2048^2, 1024^2 + 12 spot maps 1024^2..4096^2, "
                        "64-triangle scenes), 8 views (2x 720p, 1080p, 1440p, 4K), 48 jobs (cascades hard RBSM, "
                        "spots RSMSS r=0), one captured-graph replay of the autotuned plan per step",
            "fragments_per_step": bf.n_frag,
            "jobs": len(bf.jobs),
            "resident_bytes": bf.resident_bytes,
            "tuning": tune,
            "tuning_source": "fixed (--tuning)" if fixed else "autotuned",
        },
        "plain_per_view": h["plain_per_view"],
        "batched_eager": h["batched_eager"],
        "speedup_vs_plain": value / h["plain_per_view"]["fragments_per_s"],
        "p50_frame_ms": h["p50_frame_ms"],
        "p99_frame_ms": h["p99_frame_ms"],
        "bitwise_equal_to_plain": h["bitwise_equal_to_plain"],
        "roofline": {
            "kernel": kernel_instance(tune, bf.tiled_jobs) + " (batched plan, graph replay)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBPS,
            "traffic": read_traffic(khash, tune),
            "algorithmic_bytes_per_launch": frame_bytes,
            "avg_kernel_ms": h["avg_kernel_ms"],
            "kernel_source_sha": khash,
        },
    }
    del bf
    torch.cuda.empty_cache()

    if args.copy_calibration or not args.no_extras:
        out["copy_kernel_GBps"] = copy_bandwidth(torch)

    if not args.no_extras:
        out["single_view_hard"] = single_view_section(torch, rb, max(200, args.steps))
        torch.cuda.empty_cache()
        out.update(rsmss_section(torch, rb, max(100, args.steps // 2)))
        torch.cuda.empty_cache()
        out["uniform_512"] = uniform_section(torch, rb, max(500, args.steps * 5))
        torch.cuda.empty_cache()
        try:
            out["batched_per_light_radius"] = batched_radius_section(torch, rb)
        except rb.RbsmError as e:
            out["batched_per_light_radius"] = {"error": str(e)}
        torch.cuda.empty_cache()
        out["serving"] = serving_section(torch, rb)
        torch.cuda.empty_cache()
        out["raster"] = raster_section(torch, rb)
        out["composite"] = composite_section(torch, rb)
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
