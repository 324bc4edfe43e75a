"""Batched form: one launch for many uneven (view, light) jobs.

Every job's output must be bitwise the output of the plain entry point for
that job (same accuracy), under any tuning, and across graph replays.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import paper_1711_07793_amd as rb
    rb.load_library()
    return rb


@pytest.fixture(scope="module")
def workload():
    return synth.make_batched(4001, small=True)


def _device_jobs(rb, w, extra_flat=True):
    maps = [torch.from_numpy(m).cuda() for m in w["maps"]]
    jobs = []
    for j in w["jobs"]:
        f = torch.from_numpy(j["frags"]).cuda()
        out = torch.full((len(j["frags"]),), 7 if j["mode"] == 0 else -1.0,
                         dtype=torch.uint8 if j["mode"] == 0 else torch.float32, device="cuda")
        jobs.append(dict(map=maps[j["map"]], frags=f, params=j["params"], mode=j["mode"], out=out,
                         host=j))
    if extra_flat:  # a flat (no screen layout) job and a tiny ragged one
        c = synth.make_config(1, 1007, small=True)
        m1 = torch.from_numpy(c["map"]).cuda()
        f1 = torch.from_numpy(c["frags"]).cuda()
        jobs.append(dict(map=m1, frags=f1, params=c["params"], mode=1,
                         out=torch.empty(len(c["frags"]), dtype=torch.float32, device="cuda"),
                         host=dict(frags=c["frags"], params=c["params"], mode=1, map_np=c["map"])))
        jobs.append(dict(map=m1, frags=f1[:37].contiguous(), params=c["params"], mode=0,
                         out=torch.empty(37, dtype=torch.uint8, device="cuda"),
                         host=dict(frags=c["frags"][:37], params=c["params"], mode=0, map_np=c["map"])))
    return maps, jobs


def _plain(rb, j):
    if j["mode"] == 0:
        return rb.rbsm_visibility(j["map"], j["frags"], j["params"]).cpu().numpy()
    return rb.rsmss_visibility(j["map"], j["frags"], j["params"]).cpu().numpy()


# 48 jobs with tiles: job records in the kernel arguments; 50: device job tables
LAYOUTS = pytest.mark.parametrize("extra_flat", [False, True], ids=["48jobs_args", "50jobs_tables"])


@LAYOUTS
def test_batched_equals_plain_per_job(rb, workload, extra_flat):
    maps, jobs = _device_jobs(rb, workload, extra_flat)
    plan = rb.Plan(jobs)
    assert plan.fragments == sum(j["frags"].numel() // 3 for j in jobs)
    plan.launch()
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        assert np.array_equal(j["out"].cpu().numpy(), _plain(rb, j)), k
    plan.close()


def test_a_job_beyond_the_32_bit_index_form(rb, workload):
    """A plan whose jobs include one too large for the 32-bit index form
    (2^28 fragments in a 4096-pixel-wide view) runs with device job tables
    and the 64-bit form: every job's output is bitwise the plain call's."""
    maps, jobs = _device_jobs(rb, workload, extra_flat=False)
    jobs = jobs[:6]
    c = synth.make_config(1, 1025, small=True)
    m1 = torch.from_numpy(c["map"]).cuda()
    n = 1 << 28
    g = torch.Generator(device="cuda").manual_seed(25)
    f = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    f[:, 0].uniform_(-0.02, 1.02, generator=g)
    f[:, 1].uniform_(-0.02, 1.02, generator=g)
    f[:, 2].uniform_(0.3, 0.95, generator=g)
    jobs.append(dict(map=m1, frags=f, params=dict(c["params"], view_width=4096), mode=0,
                     out=torch.empty(n, dtype=torch.uint8, device="cuda")))
    plan = rb.Plan(jobs)
    plan.launch()
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        assert np.array_equal(j["out"].cpu().numpy(), _plain(rb, j)), k
    plan.close()
    del f, jobs
    torch.cuda.empty_cache()


def test_batched_against_oracle_on_a_few_jobs(rb, workload):
    maps, jobs = _device_jobs(rb, workload, extra_flat=False)
    plan = rb.Plan(jobs)
    plan.launch()
    torch.cuda.synchronize()
    for j in jobs[:6]:
        h = j["host"]
        m = workload["maps"][h["map"]]
        got = j["out"].cpu().numpy()
        if h["mode"] == 0:
            assert np.array_equal(got, oracle.rbsm_hard(m, h["frags"], h["params"]))
        else:
            assert np.max(np.abs(got - oracle.rsmss(m, h["frags"], h["params"]))) <= 1e-5


@LAYOUTS
def test_autotune_and_tunings_never_change_results(rb, workload, extra_flat):
    maps, jobs = _device_jobs(rb, workload, extra_flat)
    plan = rb.Plan(jobs)
    plan.launch()
    torch.cuda.synchronize()
    want = [j["out"].cpu().numpy().copy() for j in jobs]
    tunings = [rb.RbsmTuning(16, 1, 256), rb.RbsmTuning(64, 3, 4096),
               # direct reads (nothing staged), one workgroup per tile and resident
               rb.RbsmTuning(32, 1, 0, 0, 0, 0, 5), rb.RbsmTuning(64, 1, 0, 1, 0, 0, 5),
               # tiles dealt to XCDs in chunks (with a partial last round)
               rb.RbsmTuning(32, 1, 2048, xcd_chunk=0), rb.RbsmTuning(32, 1, 2048, xcd_chunk=3),
               rb.RbsmTuning(16, 2, 2048, xcd_chunk=12),
               # every walk blocking (one workgroup per tile)
               *[rb.RbsmTuning(tw, 1, 2048, 0, wf, wb, 5) for tw in (16, 64) for wf in (1, 2, 4) for wb in (4, 8)],
               # resident workgroups looping over tiles
               rb.RbsmTuning(16, 1, 2048, 1), rb.RbsmTuning(32, 2, 3072, 1), rb.RbsmTuning(64, 1, 2048, 1)]
    for t in tunings:
        plan.tuning = t
        for j in jobs:
            j["out"].fill_(3)
        plan.launch()
        torch.cuda.synchronize()
        for k, j in enumerate(jobs):
            assert np.array_equal(j["out"].cpu().numpy(), want[k]), (k, t.as_dict())
    chosen = plan.autotune(reps=2)
    assert chosen.tile_w in (16, 32, 64)
    for j in jobs:
        j["out"].fill_(5)
    plan.launch()
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        assert np.array_equal(j["out"].cpu().numpy(), want[k]), k


@LAYOUTS
@pytest.mark.parametrize("tuning", [None, (32, 1, 2048, 1, 0, 0, 3)])  # one workgroup per tile; resident
def test_graph_replays_match_eager(rb, workload, tuning, extra_flat):
    maps, jobs = _device_jobs(rb, workload, extra_flat)
    ref = rb.Plan(jobs)
    ref.launch()
    torch.cuda.synchronize()
    want = [j["out"].cpu().numpy().copy() for j in jobs]
    ref.close()
    plan = rb.Plan(jobs) if tuning is None else rb.Plan(jobs, tuning=tuning)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    plan.capture(s)
    for rep in range(3):
        for j in jobs:  # eager work between replays
            j["out"].fill_(rep + 11)
        torch.cuda.synchronize()
        plan.launch(s)
        s.synchronize()
        for k, j in enumerate(jobs):
            assert np.array_equal(j["out"].cpu().numpy(), want[k]), (rep, k)
    # back-to-back replays (the queue counters must be clear at every start)
    for j in jobs:
        j["out"].fill_(7)
    torch.cuda.synchronize()
    for _ in range(4):
        plan.launch(s)
    s.synchronize()
    for k, j in enumerate(jobs):
        assert np.array_equal(j["out"].cpu().numpy(), want[k]), k
    plan.close()


def test_update_swaps_buffers_with_the_same_layout(rb, workload):
    maps, jobs = _device_jobs(rb, workload, extra_flat=False)
    plan = rb.Plan(jobs)
    plan.launch()
    torch.cuda.synchronize()
    want = [j["out"].cpu().numpy().copy() for j in jobs]
    jobs2 = []
    for j in jobs:
        j2 = dict(j)
        j2["out"] = torch.zeros_like(j["out"])
        j2["frags"] = j["frags"].clone()
        jobs2.append(j2)
    plan.update(jobs2)
    plan.launch()
    torch.cuda.synchronize()
    for k, j in enumerate(jobs2):
        assert np.array_equal(j["out"].cpu().numpy(), want[k]), k
    bad = [dict(jobs2[0], frags=jobs2[0]["frags"][:10].contiguous(), out=jobs2[0]["out"][:10])] + jobs2[1:]
    with pytest.raises(rb.RbsmError):
        plan.update(bad)


@LAYOUTS
def test_update_of_a_captured_plan(rb, workload, extra_flat):
    """Replays after an update use the new buffers: the plan captures again
    (its jobs travel in kernel arguments, which a graph holds by value)."""
    maps, jobs = _device_jobs(rb, workload, extra_flat)
    plan = rb.Plan(jobs)
    plan.launch()
    torch.cuda.synchronize()
    want = [j["out"].cpu().numpy().copy() for j in jobs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    plan.capture(s)
    jobs2 = []
    for j in jobs:
        j2 = dict(j)
        j2["out"] = torch.zeros_like(j["out"])
        j2["frags"] = j["frags"].clone()
        jobs2.append(j2)
    torch.cuda.synchronize()
    plan.update(jobs2)
    for j in jobs:  # the old outputs must not be written again
        j["out"].fill_(3)
    torch.cuda.synchronize()
    plan.launch(s)
    s.synchronize()
    for k in range(len(jobs)):
        assert np.array_equal(jobs2[k]["out"].cpu().numpy(), want[k]), k
        assert np.all(jobs[k]["out"].cpu().numpy() == 3), k
    plan.close()


def test_pitched_maps(rb):
    """Jobs on maps stored with row padding (pitch > width, NaN padding that
    must never be read), hard and RSMSS, in one plan: each equals the plain
    entry point and the oracle on the unpadded map."""
    c = synth.make_config(2, 2011, small=True)
    H, W = c["map"].shape
    full = torch.full((H, W + 13), float("nan"), dtype=torch.float32, device="cuda")
    full[:, :W] = torch.from_numpy(c["map"]).cuda()
    view = full[:, :W]
    f = torch.from_numpy(c["frags"]).cuda()
    n = len(c["frags"])
    jobs = [dict(map=view, frags=f, params=dict(c["params"], pitch=None), mode=0,
                 out=torch.empty(n, dtype=torch.uint8, device="cuda")),
            dict(map=view, frags=f, params=dict(c["params"], pitch=None), mode=1,
                 out=torch.empty(n, dtype=torch.float32, device="cuda"))]
    plan = rb.Plan(jobs)
    plan.launch()
    torch.cuda.synchronize()
    p = dict(c["params"], pitch=W)
    assert np.array_equal(jobs[0]["out"].cpu().numpy(), oracle.rbsm_hard(c["map"], c["frags"], p))
    soft = jobs[1]["out"].cpu().numpy()
    assert np.max(np.abs(soft.astype(np.float64) - oracle.rsmss(c["map"], c["frags"], p))) <= 1e-5
    assert np.array_equal(soft, rb.rsmss_visibility(view, f, dict(c["params"], pitch=None)).cpu().numpy())
    plan.close()


def test_full_size_workload_sampled_against_oracle(rb):
    """The batched workload at full size (16 maps up to 8192^2, 8 views up to
    4K, 66.5 M fragment evaluations) in the launch configuration the bench
    times (autotuned): sampled fragments of every job against the oracle."""
    w = synth.make_batched(4001)
    maps, jobs = _device_jobs(rb, w, extra_flat=False)
    plan = rb.Plan(jobs)
    plan.autotune(reps=1)
    plan.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(4002)
    for k, j in enumerate(jobs):
        h = j["host"]
        n = len(h["frags"])
        idx = np.sort(rng.choice(n, min(n, 1500), replace=False))
        got = j["out"].cpu().numpy()[idx]
        f = np.ascontiguousarray(h["frags"][idx])
        m = w["maps"][h["map"]]
        p = dict(h["params"], pitch=m.shape[1])
        if j["mode"] == 0:
            want = oracle.rbsm_hard(m, f, p)
            bad = np.nonzero(got != want)[0]
            assert len(bad) <= max(0, int(1e-5 * len(want))), (k, len(bad))
        else:
            want = oracle.rsmss(m, f, p)
            assert np.max(np.abs(got.astype(np.float64) - want)) <= 1e-5, k
    plan.close()
    del maps, jobs
    torch.cuda.empty_cache()


def test_rpcf_jobs_in_the_plan(rb, workload):
    """RSMSS jobs with a kernel radius (each spot light its own r) run the
    box filter inside the plan: bitwise the plain rsmss_visibility result,
    eager and from graph replays, and within 1e-5 of the oracle."""
    maps, jobs = _device_jobs(rb, workload)
    radii = {}
    for k, j in enumerate(jobs):
        if j["mode"] == 1:
            r = radii.setdefault(id(j["map"]), 1 + (k % 6))
            j["params"] = dict(j["params"], kernel_radius=r)
    assert len(set(radii.values())) > 1
    want = [_plain(rb, j) for j in jobs]
    plan = rb.Plan(jobs)
    plan.launch()
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        assert np.array_equal(j["out"].cpu().numpy(), want[k]), k
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    plan.capture(s)
    for rep in range(3):
        for j in jobs:
            j["out"].fill_(9)
        torch.cuda.synchronize()
        plan.launch(s)
        s.synchronize()
        for k, j in enumerate(jobs):
            assert np.array_equal(j["out"].cpu().numpy(), want[k]), (rep, k)
    rng = np.random.default_rng(11)
    for k, j in enumerate(jobs):
        if j["mode"] != 1:
            continue
        h = j["host"]
        m = h.get("map_np")
        if m is None:
            m = workload["maps"][h["map"]]
        n = len(h["frags"])
        idx = np.sort(rng.choice(n, min(n, 400), replace=False))
        f = np.ascontiguousarray(h["frags"][idx])
        got = j["out"].cpu().numpy()[idx]
        ref = oracle.rsmss(m, f, dict(j["params"], pitch=m.shape[1]))
        assert np.max(np.abs(got.astype(np.float64) - ref)) <= 1e-5, k
    # a radius change is a layout change: update rejects it
    bad = [dict(j) for j in jobs]
    for j in bad:
        if j["mode"] == 1:
            j["params"] = dict(j["params"], kernel_radius=j["params"]["kernel_radius"] + 1)
            break
    with pytest.raises(rb.RbsmError):
        plan.update(bad)
    plan.close()


@pytest.mark.parametrize("copies", [1, 9], ids=["args", "tables"])
def test_mixed_job_order_empty_and_rpcf_jobs(rb, copies):
    """Jobs whose modes alternate, with empty jobs and RPCF jobs between them:
    the plan launches the RSMSS jobs' tiles first, the allocation-free entry
    point in job order; every output is bitwise the plain call's (one plan of
    6 jobs, kernel-argument records; nine copies, 54 jobs, device tables)."""
    c2 = synth.make_config(2, 2011, small=True)
    c3 = synth.make_config(3, 3011, small=True)
    m2, f2 = torch.from_numpy(c2["map"]).cuda(), torch.from_numpy(c2["frags"]).cuda()
    m3, f3 = torch.from_numpy(c3["map"]).cuda(), torch.from_numpy(c3["frags"]).cuda()

    def job(mode, m, f, params, n=None):
        f = f if n is None else f[:n].contiguous()
        out = torch.full((f.shape[0],), 7 if mode == 0 else -1.0,
                         dtype=torch.uint8 if mode == 0 else torch.float32, device="cuda")
        return dict(map=m, frags=f, params=params, mode=mode, out=out)

    jobs = []
    for _ in range(copies):
        jobs += [job(0, m2, f2, c2["params"]),
                 job(1, m3, f3, dict(c3["params"], kernel_radius=0), n=0),
                 job(1, m3, f3, dict(c3["params"], kernel_radius=0)),
                 job(1, m3, f3, dict(c3["params"], kernel_radius=2), n=5000),
                 job(0, m2, f2, c2["params"], n=0),
                 job(1, m2, f2, dict(c2["params"], kernel_radius=0), n=777)]
    want = [_plain(rb, j) for j in jobs]
    plan = rb.Plan(jobs)
    plan.launch()
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        assert np.array_equal(j["out"].cpu().numpy(), want[k]), ("plan", k)
    plan.close()
    for j in jobs:
        j["out"].fill_(3)
    rb.batch_launch_noalloc(jobs)
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        assert np.array_equal(j["out"].cpu().numpy(), want[k]), ("noalloc", k)
