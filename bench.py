"""Benchmark of the RBSM per-fragment shadow pass on one MI355X.

One step = one plain per-view pass of the hot path over one frame: hard RBSM
(silhouette recovery) of 1920x1080 perspective-camera fragments against a
2048^2 float32 depth map of 64 random triangles over a tilted receiver,
MAXDIST 32, depth bias 1e-4 (the paper's 2048^2 / 1080p hard-shadow
operating point, Table 3, on synthetic scenes).  Frames rotate over at least
512 MB of distinct device buffers so their bytes come from HBM, not from the
256 MB last-level cache.  All inputs are resident on the device before timing.

Prints ONE JSON line.  Besides the headline value it reports the dominant
kernel's roofline (algorithmic bytes / kernel time from HIP events recorded
around every launch on the launch stream), the RSMSS pass at 3840x2160 on a
4096^2 map with the thin-bar fence, the plain shadow-mapping pass of the same
frames, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shaded fragments/sec (RBSM, RSMSS) batched vs plain per-view; p99 frame latency"
PEAK_HBM_GBPS = 8000.0
ROTATE_BYTES = 512 << 20
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "tile_kernel_hard_tri64_map2048_1080p_traffic.md")


def kernel_source_hash() -> str:
    """Hash of the sources that define the hard-pass kernel (tile pass and the
    per-fragment device helpers)."""
    h = hashlib.sha256()
    for rel in ("paper_1711_07793_amd/csrc/tile_pass.hpp", "paper_1711_07793_amd/csrc/rbsm_device.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_hash: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on a different kernel source."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    vals = {}
    for line in open(PROFILE_TRAFFIC):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha") != kernel_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(steps):
        a = args[k % nslot]
        fn(a[0], a[1], a[2], a[3], a[4], sh)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_ms = ev0.elapsed_time(ev1) / steps
    used = [k % nslot for k in range(steps)]
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


def batched_section(torch, rb, frames_timed: int = 20):
    """The batched workload (16 maps, 8 views, 48 jobs of uneven size) run as
    plain per-view launches (one call per job, frame-synchronised), as one
    batched launch per frame, and as one graph replay per frame."""
    import synth
    w = synth.make_batched(4001)
    maps = [torch.from_numpy(m).cuda() for m in w["maps"]]
    jobs = []
    for j in w["jobs"]:
        f = torch.from_numpy(j["frags"]).cuda()
        out = torch.empty(len(j["frags"]), dtype=torch.uint8 if j["mode"] == 0 else torch.float32, device="cuda")
        jobs.append(dict(map=maps[j["map"]], frags=f, params=j["params"], mode=j["mode"], out=out))
    n_frag = sum(j["frags"].numel() // 3 for j in jobs)
    lib = rb.load_library()
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    cparams = [rb.Params(**j["params"]).to_c() for j in jobs]

    def plain_frame():
        for j, p in zip(jobs, cparams):
            fn = lib.rbsm_visibility if j["mode"] == 0 else lib.rsmss_visibility
            st = fn(j["map"].data_ptr(), j["frags"].data_ptr(), j["frags"].numel() // 3, ctypes.byref(p),
                    j["out"].data_ptr(), sh)
            assert st == 0, rb.rbsm_last_error()

    def run(frame_fn, sync_fn):
        for _ in range(3):
            frame_fn()
        sync_fn()
        lat = []
        t0 = time.perf_counter()
        for _ in range(frames_timed):
            a = time.perf_counter()
            frame_fn()
            sync_fn()
            lat.append((time.perf_counter() - a) * 1e3)
        wall = time.perf_counter() - t0
        lat = np.array(lat)
        return {"fragments_per_s": n_frag * frames_timed / wall, "p50_frame_ms": float(np.percentile(lat, 50)),
                "p99_frame_ms": float(np.percentile(lat, 99))}

    plain = run(plain_frame, torch.cuda.synchronize)
    want = [j["out"].clone() for j in jobs]
    plan = rb.Plan(jobs)
    tune = plan.autotune(reps=3)
    for j in jobs:
        j["out"].fill_(0)
    plan.launch()
    torch.cuda.synchronize()
    equal = all(torch.equal(j["out"], wv) for j, wv in zip(jobs, want))
    batched = run(plan.launch, torch.cuda.synchronize)
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    plan.capture(s)
    graph = run(lambda: plan.launch(s), s.synchronize)
    plan.close()
    return {
        "workload": "16 maps (cascades 8192^2..1024^2 + 12 spot maps 1024^2..4096^2), 8 views 720p..4K, "
                    f"{len(jobs)} jobs (cascades hard, spots RSMSS r=0)",
        "fragments_per_frame": n_frag,
        "plain_per_view": plain,
        "batched": batched,
        "batched_graph": graph,
        "speedup_vs_plain": batched["fragments_per_s"] / plain["fragments_per_s"],
        "graph_speedup_vs_plain": graph["fragments_per_s"] / plain["fragments_per_s"],
        "tuning": {"tile_w": tune.tile_w, "apron": tune.apron, "lds_cap": tune.lds_cap},
        "bitwise_equal_to_plain": bool(equal),
    }


def cpu_baseline(frames: Frames, budget_s: float):
    """Oracle (single-threaded C) on a bounded sample of the same frames."""
    import oracle
    done = 0
    t0 = time.perf_counter()
    k = 0
    while True:
        h = frames.host[k % len(frames.host)]
        oracle.rbsm_hard(h["map"], h["frags"], h["params"])
        done += len(h["frags"])
        k += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="fragments/s", cores=1, kind="oracle",
                sample=f"{k} full frames ({done} fragments) of the same workload, 5 scenes cycled, "
                       f"{dt:.1f} s single-threaded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(every fragment/light evaluation is independent; multi-GPU sharding is described "
              "in the design notes but not run).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1711_07793_amd as rb

    lib = rb.load_library()
    torch.cuda.init()

    # ---- headline: hard RBSM, 2048^2 map, 1920x1080 fragments -----------
    frames = Frames(torch, 2, [2001, 2002, 2003, 2004, 2005], ROTATE_BYTES, "hard", torch.uint8)
    params = frames.params
    wall, avg_kernel_ms, used = time_pass(torch, rb, lib, "rbsm_visibility", frames, params, args.steps,
                                          args.warmup)
    ms_per_step = wall * 1e3 / args.steps
    value = frames.n * args.steps / wall
    per_frame_bytes = algorithmic_bytes(torch, rb, frames, params, 0, 1)
    slot_scene = [s[0] for s in frames.slots]
    bytes_per_launch = float(np.mean([per_frame_bytes[slot_scene[u]] for u in used]))
    p50_ms, p99_ms = launch_latency(torch, rb, lib, "rbsm_visibility", frames, params, 500)
    achieved = bytes_per_launch / (avg_kernel_ms * 1e-3) / 1e9
    khash = kernel_source_hash()
    traffic = read_traffic(khash)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "fragments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "hard RBSM, 2048x2048 f32 map of 64 random triangles over a tilted receiver, "
                        "1920x1080 perspective fragments, MAXDIST 32, bias 1e-4, plain per-view launch",
            "fragments_per_step": frames.n,
            "frames_rotated": len(frames.slots),
            "resident_bytes": frames.bytes_resident,
        },
        "roofline": {
            "kernel": "tile_kernel<true, 32> (hard pass)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBPS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_kernel_ms": avg_kernel_ms,
            "kernel_source_sha": khash,
        },
        "p50_frame_ms": p50_ms,
        "p99_frame_ms": p99_ms,
    }

    if args.copy_calibration or not args.no_extras:
        out["copy_kernel_GBps"] = copy_bandwidth(torch)

    if not args.no_extras:
        # plain shadow mapping of the same frames (the paper's baseline pass)
        w_sm, a_sm, _ = time_pass(torch, rb, lib, "sm_visibility", frames, params, max(200, args.steps // 4), 20)
        out["plain_sm"] = {"fragments_per_s": frames.n * max(200, args.steps // 4) / w_sm,
                           "avg_kernel_ms": a_sm}
        del frames
        torch.cuda.empty_cache()
        # RSMSS at 3840x2160 on a 4096^2 fenced scene, radius 0 (Listing 5 exactly)
        fr3 = Frames(torch, 3, [3001, 3002, 3003], ROTATE_BYTES, "rsmss", torch.float32)
        p3 = dict(fr3.params, kernel_radius=0)
        steps3 = max(100, args.steps // 10)
        w3, a3, used3 = time_pass(torch, rb, lib, "rsmss_visibility", fr3, p3, steps3, 10)
        b3 = algorithmic_bytes(torch, rb, fr3, p3, 1, 4)
        sc3 = [s[0] for s in fr3.slots]
        bpl3 = float(np.mean([b3[sc3[u]] for u in used3]))
        out["rsmss"] = {
            "workload": "RSMSS r=0, 4096x4096 map of 256 triangles + thin-bar fence, 3840x2160 fragments, "
                        "MAXDIST 16",
            "fragments_per_s": fr3.n * steps3 / w3,
            "ms_per_step": w3 * 1e3 / steps3,
            "avg_kernel_ms": a3,
            "achieved_GBps": bpl3 / (a3 * 1e-3) / 1e9,
            "algorithmic_bytes_per_launch": bpl3,
        }
        # RPCF at the light's own kernel radius (the same frames)
        r3 = fr3.host[0]["light_radius"]
        pr = dict(fr3.params, kernel_radius=r3)
        steps_r = max(20, args.steps // 100)
        wr, ar, _ = time_pass(torch, rb, lib, "rsmss_visibility", fr3, pr, steps_r, 3)
        out["rpcf"] = {
            "workload": f"RPCF radius {r3} ({(2 * r3 + 1) ** 2} RSMSS terms per fragment) on the RSMSS frames",
            "kernel_radius": r3,
            "fragments_per_s": fr3.n * steps_r / wr,
            "ms_per_step": wr * 1e3 / steps_r,
            "avg_kernel_ms": ar,
            "terms_per_s": fr3.n * (2 * r3 + 1) ** 2 / (ar * 1e-3),
        }
        del fr3
        torch.cuda.empty_cache()
        out["batched"] = batched_section(torch, rb)
        torch.cuda.empty_cache()
        frames = Frames.__new__(Frames)  # host frames for the CPU leg
        import synth
        frames.host = [synth.make_config(2, s) for s in (2001, 2002, 2003, 2004, 2005)]
        out["cpu_baseline"] = cpu_baseline(frames, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
