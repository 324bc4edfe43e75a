"""Serving form and multi-light compositing on the GPU.

Every per-light result of the engine must be bitwise the plain entry point's,
every composite bitwise the composite entry point's on those results, and all
of it must be the same whether a request runs alone or mixed with others under
a tight HBM budget.  A sample is checked against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

SOFT_TOL = 1e-5


@pytest.fixture(scope="module")
def rb():
    import paper_1711_07793_amd as rb
    rb.load_library()
    return rb


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def world(rb):
    """6 resident lights (random-triangle maps 128^2..512^2) and, for each
    light, camera fragments of 3 small views (device-resident)."""
    sizes = [128, 256, 512, 128, 256, 512]
    views = [(160, 90), (240, 135), (320, 180)]
    lights, frags = [], {}
    for li, S in enumerate(sizes):
        sc = synth.triangle_scene(7100 + li, S, S, 48, fence=(li % 3 == 2))
        m = sc.raster()
        lights.append(m)
        for vi, (w, h) in enumerate(views):
            frags[(li, vi)] = sc.camera_fragments(7200 + 10 * li + vi, w, h)
    dev_maps = [torch.from_numpy(m).cuda() for m in lights]
    dev_frags = {k: torch.from_numpy(v).cuda() for k, v in frags.items()}
    rng = np.random.default_rng(7300)
    reqs = []
    for q in range(24):
        vi = int(rng.integers(0, 3))
        nl = int(rng.integers(1, 5))
        ls = rng.choice(6, size=nl, replace=False)
        L = []
        for li in ls:
            mode = int(li % 2)
            radius = 2 if (mode == 1 and q % 5 == 0) else 0
            L.append(dict(light=int(li), mode=mode, depth_bias=1e-4, max_dist=16 if li < 3 else 24,
                          kernel_radius=radius, weight=float(np.float32(rng.uniform(0.1, 1.0)))))
        reqs.append(dict(view=vi, lights=L))
    return dict(maps=lights, dev_maps=dev_maps, frags=frags, dev_frags=dev_frags, views=views, reqs=reqs)


def _outs(world, req, where="pinned"):
    """Result buffers: pinned host, pageable host, or device (written in place)."""
    w, h = world["views"][req["view"]]
    n = w * h

    def buf(dtype):
        if where == "device":
            return torch.full((n,), 7, dtype=dtype, device="cuda")
        t = torch.empty(n, dtype=dtype)
        return t.pin_memory() if where == "pinned" else t

    outs = [buf(torch.uint8 if L["mode"] == 0 else torch.float32) for L in req["lights"]]
    return n, w, outs, buf(torch.float32)


def _submit(eng, ids, world, req, outs, comp, host_frags=None):
    w, h = world["views"][req["view"]]
    lights = []
    for L, o in zip(req["lights"], outs):
        f = world["dev_frags"][(L["light"], req["view"])] if host_frags is None else \
            host_frags[(L["light"], req["view"])]
        lights.append(dict(L, light=ids[L["light"]], frags=f, out=o))
    return eng.submit(w * h, lights, view_width=w, composite=comp)


def _run(rb, world, budget, max_inflight, burst, where="pinned", host_frags=None):
    eng = rb.Engine(budget, max_inflight)
    ids = [eng.add_light(m) for m in world["dev_maps"]]
    results = []
    tickets = []
    for req in world["reqs"]:
        n, w, outs, comp = _outs(world, req, where)
        t = _submit(eng, ids, world, req, outs, comp, host_frags)
        if burst:
            tickets.append(t)
        else:
            assert eng.wait(t, 60000) is not None
        results.append((outs, comp))
    for t in tickets:
        assert eng.wait(t, 60000) is not None
    st = eng.stats()
    eng.close()
    return [([o.cpu().numpy().copy() for o in outs], comp.cpu().numpy().copy()) for outs, comp in results], st


def _plain(rb, world, req):
    w, h = world["views"][req["view"]]
    outs = []
    for L in req["lights"]:
        m = world["dev_maps"][L["light"]]
        f = world["dev_frags"][(L["light"], req["view"])]
        p = dict(width=m.shape[1], height=m.shape[0], depth_bias=L["depth_bias"], max_dist=L["max_dist"],
                 kernel_radius=L["kernel_radius"], view_width=w)
        outs.append(rb.rbsm_visibility(m, f, p) if L["mode"] == 0 else rb.rsmss_visibility(m, f, p))
    comp = rb.rbsm_composite(outs, [L["mode"] for L in req["lights"]], [L["weight"] for L in req["lights"]])
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], comp.cpu().numpy()


def test_composite_entry_point_matches_oracle(rb):
    n = 100003
    a = synth.uniform_floats(41, n)
    b = synth.uniform_floats(42, n)
    h = (synth.uniform_floats(43, n) < 0.5).astype(np.uint8)
    w = [0.7, 0.2, 0.1]
    want = oracle.composite([a, h, b], w)
    got = rb.rbsm_composite([torch.from_numpy(a).cuda(), torch.from_numpy(h).cuda(), torch.from_numpy(b).cuda()],
                            [1, 0, 1], w).cpu().numpy()
    assert np.array_equal(got, want)
    one = rb.rbsm_composite([torch.from_numpy(h).cuda()], [0], [1.0]).cpu().numpy()
    assert np.array_equal(one, h.astype(np.float32))
    # buffers that do not start aligned: fragment by fragment, the same sums
    # (s = 4: aligned again, 4 fragments per load)
    for s in (1, 2, 3, 4):
        da, dh = torch.from_numpy(a).cuda(), torch.from_numpy(h).cuda()
        out = torch.zeros(n + 4, dtype=torch.float32, device="cuda")
        got = rb.rbsm_composite([da[s:], dh[s:], da[:n - s]], [1, 0, 1], w, out=out[s:n]).cpu().numpy()
        assert np.array_equal(got, oracle.composite([a[s:], h[s:], a[:n - s]], w)), s
        assert np.all(out[:s].cpu().numpy() == 0) and np.all(out[n:].cpu().numpy() == 0)


@pytest.mark.parametrize("n_lights", [4, 8])
def test_composite_full_4k_view(rb, n_lights):
    """A whole 3840 x 2160 view, as the benchmark composites it: every
    fragment bit-equal to the oracle, hard and RSMSS lights alternating."""
    n = 3840 * 2160
    say(f"composite 4K lights={n_lights}")
    vis, modes = [], []
    for l in range(n_lights):
        u = synth.uniform_floats(500 + l, n)
        if l % 2 == 0:
            vis.append((u < 0.5).astype(np.uint8))
            modes.append(0)
        else:
            vis.append(u)
            modes.append(1)
    w = list(synth.uniform_floats(600 + n_lights, n_lights) / n_lights)
    got = rb.rbsm_composite([torch.from_numpy(v).cuda() for v in vis], modes, w).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), oracle.composite(vis, w).view(np.uint32))


def test_alone_and_in_the_mix_are_identical(rb, world):
    say("serving: alone")
    alone, st_a = _run(rb, world, budget=256 << 20, max_inflight=8, burst=False)
    # a budget that holds only a few requests' results at a time forces
    # admission waits, several requests per step and overlapping steps
    say("serving: mix")
    mix, st_m = _run(rb, world, budget=6 << 20, max_inflight=6, burst=True)
    assert st_a["completed"] == st_m["completed"] == len(world["reqs"])
    assert st_m["launches"] < len(world["reqs"])          # requests were batched together
    assert st_m["arena_peak_bytes"] <= st_m["arena_bytes"]
    assert 0 < st_m["inflight_peak_bytes"] <= 6 << 20        # working sets held within the budget
    for k, ((oa, ca), (om, cm)) in enumerate(zip(alone, mix)):
        for x, y in zip(oa, om):
            assert np.array_equal(x, y), k
        assert np.array_equal(ca, cm), k
    # results written in place on the device (no staging) and to pageable host
    # memory: the same values again
    say("serving: device and pageable destinations")
    dev, st_d = _run(rb, world, budget=5 << 20, max_inflight=6, burst=True, where="device")
    assert st_d["arena_peak_bytes"] == 0                  # nothing staged
    page, _ = _run(rb, world, budget=6 << 20, max_inflight=6, burst=True, where="pageable")
    for k in range(len(alone)):
        for x, y, z in zip(alone[k][0], dev[k][0], page[k][0]):
            assert np.array_equal(x, y) and np.array_equal(x, z), k
        assert np.array_equal(alone[k][1], dev[k][1]) and np.array_equal(alone[k][1], page[k][1]), k
    say("serving: plain entry points")
    for k, req in enumerate(world["reqs"]):
        po, pc = _plain(rb, world, req)
        for x, y in zip(alone[k][0], po):
            assert np.array_equal(x, y), k
        assert np.array_equal(alone[k][1], pc), k


def test_engine_results_against_oracle(rb, world):
    eng = rb.Engine(64 << 20, 4)
    ids = [eng.add_light(m) for m in world["dev_maps"]]
    for req in world["reqs"][:6]:
        n, w, outs, comp = _outs(world, req)
        t = _submit(eng, ids, world, req, outs, comp)
        assert eng.wait(t, 60000) is not None
        want = []
        for L, o in zip(req["lights"], outs):
            m = world["maps"][L["light"]]
            f = world["frags"][(L["light"], req["view"])]
            p = dict(width=m.shape[1], height=m.shape[0], pitch=m.shape[1], depth_bias=L["depth_bias"],
                     max_dist=L["max_dist"], kernel_radius=L["kernel_radius"])
            if L["mode"] == 0:
                v = oracle.rbsm_hard(m, f, p)
                assert np.array_equal(o.numpy(), v)
            else:
                v = oracle.rsmss(m, f, p)
                assert np.max(np.abs(o.numpy().astype(np.float64) - v)) <= SOFT_TOL
            want.append(v)
        wc = oracle.composite(want, [L["weight"] for L in req["lights"]])
        tol = SOFT_TOL * sum(abs(L["weight"]) for L in req["lights"]) + 1e-6
        assert np.max(np.abs(comp.numpy().astype(np.float64) - wc)) <= tol
    eng.close()


def test_engine_rejections_and_empty_request(rb, world):
    eng = rb.Engine(1 << 20, 2)
    lid = eng.add_light(world["dev_maps"][0])
    f = world["dev_frags"][(0, 2)]
    n = f.numel() // 3
    with pytest.raises(rb.RbsmError):   # results alone exceed the budget
        eng.submit(n, [dict(light=lid, mode=1, frags=f)] * 8)
    with pytest.raises(rb.RbsmError):   # unknown light
        eng.submit(n, [dict(light=99, mode=0, frags=f)])
    with pytest.raises(rb.RbsmError):   # radius in hard mode
        eng.submit(n, [dict(light=lid, mode=0, frags=f, kernel_radius=2)])
    with pytest.raises(rb.RbsmError):
        eng.wait(12345, 10)
    with pytest.raises(rb.RbsmError):   # a device result buffer over the fragments
        eng.submit(n, [dict(light=lid, mode=1, frags=f, out=f.view(-1)[:n])])
    empty = torch.empty(0, 3, dtype=torch.float32, device="cuda")
    t = eng.submit(0, [dict(light=lid, mode=0, frags=empty)])
    assert eng.wait(t, 10000) is not None
    eng.close()


def test_poisson_arrivals_complete(rb, world):
    """Requests arriving while others run: all complete, latencies positive."""
    import threading
    import time
    eng = rb.Engine(8 << 20, 16)
    ids = [eng.add_light(m) for m in world["dev_maps"]]
    rng = np.random.default_rng(7400)
    gaps = rng.exponential(0.0005, size=len(world["reqs"]))
    tickets, bufs = [], []

    def producer():
        for req, g in zip(world["reqs"], gaps):
            time.sleep(g)
            n, w, outs, comp = _outs(world, req)
            bufs.append((outs, comp))
            tickets.append(_submit(eng, ids, world, req, outs, comp))

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    lat = [eng.wait(t, 60000) for t in tickets]
    assert all(x is not None and x > 0 for x in lat)
    st = eng.stats()
    assert st["completed"] == len(world["reqs"]) and st["queued"] == 0 and st["inflight"] == 0
    eng.close()


def test_pitched_light(rb, world):
    """A light registered as a row-padded view (pitch > width, NaN padding):
    the engine's results equal the plain entry point's on the same view."""
    m = world["maps"][1]
    H, W = m.shape
    full = torch.full((H, W + 7), float("nan"), dtype=torch.float32, device="cuda")
    full[:, :W] = torch.from_numpy(m).cuda()
    view = full[:, :W]
    eng = rb.Engine(64 << 20, 4)
    lid = eng.add_light(view)
    w, h = world["views"][2]
    f = world["dev_frags"][(1, 2)]
    outs = [torch.empty(w * h, dtype=torch.uint8, device="cuda"), torch.empty(w * h, dtype=torch.float32,
                                                                               device="cuda")]
    t = eng.submit(w * h, [dict(light=lid, mode=0, frags=f, out=outs[0], max_dist=16, depth_bias=1e-4),
                           dict(light=lid, mode=1, frags=f, out=outs[1], max_dist=16, depth_bias=1e-4)],
                   view_width=w)
    assert eng.wait(t, 60000) is not None
    p = dict(width=W, height=H, depth_bias=1e-4, max_dist=16, view_width=w)
    assert np.array_equal(outs[0].cpu().numpy(), rb.rbsm_visibility(view, f, p).cpu().numpy())
    assert np.array_equal(outs[1].cpu().numpy(), rb.rsmss_visibility(view, f, p).cpu().numpy())
    hp = dict(width=W, height=H, pitch=W, depth_bias=1e-4, max_dist=16, kernel_radius=0)
    assert np.array_equal(outs[0].cpu().numpy(), oracle.rbsm_hard(m, world["frags"][(1, 2)], hp))
    eng.close()


def test_full_size_requests_sampled_against_oracle(rb):
    """Serving at full size: resident lights of 1024^2..8192^2 and views of
    720p..4K, as the bench runs them (device destinations, a composite per
    request); sampled fragments of every light and of the composite against
    the oracle."""
    sizes = [1024, 4096, 8192, 2048]
    views = [(1280, 720), (1920, 1080), (3840, 2160)]
    scenes = [synth.triangle_scene(7500 + li, S, S, 64) for li, S in enumerate(sizes)]
    maps = [sc.raster() for sc in scenes]
    eng = rb.Engine(4 << 30, 8)
    ids = [eng.add_light(torch.from_numpy(m).cuda()) for m in maps]
    rng = np.random.default_rng(7501)
    reqs = [(0, [0, 2]), (1, [1, 3, 2]), (2, [2, 0]), (2, [3]), (1, [0, 1, 2, 3])]
    for vi, ls in reqs:
        w, h = views[vi]
        n = w * h
        host_frags = [scenes[li].camera_fragments(7600 + 10 * li + vi, w, h) for li in ls]
        lights, outs = [], []
        for k, li in enumerate(ls):
            mode = li % 2
            o = torch.empty(n, dtype=torch.uint8 if mode == 0 else torch.float32, device="cuda")
            outs.append(o)
            lights.append(dict(light=ids[li], mode=mode, frags=torch.from_numpy(host_frags[k]).cuda(),
                               depth_bias=1e-4, max_dist=16, weight=float(np.float32(0.25 + 0.5 * k / len(ls))),
                               out=o))
        comp = torch.empty(n, dtype=torch.float32, device="cuda")
        t = eng.submit(n, lights, view_width=w, composite=comp)
        assert eng.wait(t, 60000) is not None
        idx = np.sort(rng.choice(n, 1200, replace=False))
        vis = []
        for k, li in enumerate(ls):
            m = maps[li]
            f = np.ascontiguousarray(host_frags[k][idx])
            p = dict(width=m.shape[1], height=m.shape[0], pitch=m.shape[1], depth_bias=1e-4, max_dist=16,
                     kernel_radius=0)
            got = outs[k].cpu().numpy()[idx]
            if li % 2 == 0:
                v = oracle.rbsm_hard(m, f, p)
                assert np.array_equal(got, v), (vi, li)
            else:
                v = oracle.rsmss(m, f, p)
                assert np.max(np.abs(got.astype(np.float64) - v)) <= SOFT_TOL, (vi, li)
            vis.append(v)
        wc = oracle.composite(vis, [L["weight"] for L in lights])
        tol = SOFT_TOL * sum(L["weight"] for L in lights) + 1e-6
        assert np.max(np.abs(comp.cpu().numpy()[idx].astype(np.float64) - wc)) <= tol, vi
    eng.close()


def test_host_fragments_uploaded_under_a_tight_budget(rb, world):
    """Fragments in pinned host memory are uploaded into the engine's arena; a
    budget of about 1.5 of the largest request's working set makes requests
    wait for earlier ones' fragments and results to leave before theirs are
    uploaded.  Every result equals the device-resident run, bitwise."""
    say("serving: device-resident fragments")
    ref, _ = _run(rb, world, budget=256 << 20, max_inflight=8, burst=True)
    host = {k: torch.from_numpy(v.copy()).pin_memory() for k, v in world["frags"].items()}
    say("serving: host fragments, tight budget")
    got, st = _run(rb, world, budget=6 << 20, max_inflight=8, burst=True, host_frags=host)
    assert st["completed"] == len(world["reqs"])
    assert st["uploaded_bytes"] == sum(12 * world["views"][r["view"]][0] * world["views"][r["view"]][1] *
                                       len(r["lights"]) for r in world["reqs"])
    assert 0 < st["inflight_peak_bytes"] <= 6 << 20
    for k in range(len(ref)):
        for x, y in zip(ref[k][0], got[k][0]):
            assert np.array_equal(x, y), k
        assert np.array_equal(ref[k][1], got[k][1]), k
    # pageable host fragments: the same
    page = {k: torch.from_numpy(v.copy()) for k, v in world["frags"].items()}
    got2, _ = _run(rb, world, budget=6 << 20, max_inflight=4, burst=True, where="device", host_frags=page)
    for k in range(len(ref)):
        for x, y in zip(ref[k][0], got2[k][0]):
            assert np.array_equal(x, y), k


def test_requests_wait_for_their_producer_stream(rb, world):
    """Fragments and output buffers produced asynchronously on a side stream:
    the request's kernels wait for that stream's work before the submit."""
    eng = rb.Engine(256 << 20, 8)
    ids = [eng.add_light(m) for m in world["dev_maps"]]
    side = torch.cuda.Stream()
    big = torch.randn(4096, 4096, device="cuda")
    for req in world["reqs"][:6]:
        w, h = world["views"][req["view"]]
        n = w * h
        with torch.cuda.stream(side):
            busy = big @ big                       # keeps the side stream busy a while
            lights, outs = [], []
            for L in req["lights"]:
                src = world["dev_frags"][(L["light"], req["view"])]
                f = torch.empty_like(src)
                f.copy_(src)                       # produced on the side stream
                o = torch.full((n,), 3 if L["mode"] == 0 else -3.0,
                               dtype=torch.uint8 if L["mode"] == 0 else torch.float32, device="cuda")
                outs.append(o)
                lights.append(dict(L, light=ids[L["light"]], frags=f, out=o))
        t = eng.submit(n, lights, view_width=w, stream=side)
        assert eng.wait(t, 60000) is not None
        del busy
        po, _ = _plain(rb, world, req)
        for x, y in zip(outs, po):
            assert np.array_equal(x.cpu().numpy(), y)
    eng.close()


def test_abort_fails_pending_requests_cleanly(rb, world):
    """rbsm_engine_abort (forced from the host; every kernel runs normally):
    each wait returns (done before the abort, or an error after the work
    already enqueued finished), the counters drain, later submissions are
    rejected, and the engine closes."""
    eng = rb.Engine(6 << 20, 2)
    ids = [eng.add_light(m) for m in world["dev_maps"]]
    bufs = [_outs(world, req, "device") for req in world["reqs"]]
    side = torch.cuda.Stream()
    big = torch.randn(4096, 4096, device="cuda")
    with torch.cuda.stream(side):
        for _ in range(12):                # the requests' producer stream stays busy a while
            big = big @ big / 4096.0
    tickets = []
    for req, (n, w, outs, comp) in zip(world["reqs"], bufs):
        lights = [dict(L, light=ids[L["light"]], frags=world["dev_frags"][(L["light"], req["view"])], out=o)
                  for L, o in zip(req["lights"], outs)]
        tickets.append(eng.submit(n, lights, view_width=w, composite=comp, stream=side))
    eng.abort("test")
    done = failed = 0
    for t in tickets:
        try:
            assert eng.wait(t, 60000) is not None
            done += 1
        except rb.RbsmError as e:
            assert "aborted" in str(e)
            failed += 1
    assert done + failed == len(tickets) and failed > 0
    st = eng.stats()
    assert st["queued"] == 0 and st["inflight"] == 0 and st["inflight_bytes"] == 0
    n, w, outs, comp = _outs(world, world["reqs"][0], "device")
    with pytest.raises(rb.RbsmError):
        _submit(eng, ids, world, world["reqs"][0], outs, comp)
    eng.close()
    side.synchronize()
