"""The batched entry point that allocates nothing (its tables live in a
per-GPU device array of the library): called through the C ABI, its outputs
must equal those of the plan entry points bitwise, on two calls in a row,
the second with a smaller input."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import paper_1711_07793_amd as rb
    rb.load_library()
    return rb


def _jobs(rb, w, radius=False):
    maps = [torch.from_numpy(m).cuda() for m in w["maps"]]
    jobs = []
    for k, j in enumerate(w["jobs"]):
        params = dict(j["params"])
        if radius and j["mode"] == 1 and k % 3 == 0:
            params["kernel_radius"] = 2
        f = torch.from_numpy(j["frags"]).cuda()
        out = torch.full((len(j["frags"]),), 7 if j["mode"] == 0 else -1.0,
                         dtype=torch.uint8 if j["mode"] == 0 else torch.float32, device="cuda")
        jobs.append(dict(map=maps[j["map"]], frags=f, params=params, mode=j["mode"], out=out))
    return maps, jobs


def _via_plan(rb, jobs, tuning):
    want_jobs = [dict(j, out=torch.empty_like(j["out"])) for j in jobs]
    plan = rb.Plan(want_jobs, tuning=tuning)
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    return [j["out"].cpu().numpy() for j in want_jobs]


def _noalloc_c_abi(rb, jobs, tuning):
    """Call the entry point directly through the C ABI."""
    lib = rb.load_library()
    arr, keep = rb.Plan._marshal(jobs)
    t = None if tuning is None else ctypes.byref(rb.RbsmTuning(*tuning))
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.rbsm_batch_launch_noalloc(arr, len(jobs), t, ctypes.c_void_p(stream))
    assert st == 0, rb.rbsm_last_error()
    torch.cuda.synchronize()
    return [j["out"].cpu().numpy() for j in jobs]


@pytest.mark.parametrize("tuning", [None, (64, 1, 2048, 0, 1, 8, 5), (32, 2, 2048, 1, 0, 0, -1)])
def test_noalloc_equals_plan_twice_then_smaller(rb, tuning):
    w = synth.make_batched(4001, small=True)
    maps, jobs = _jobs(rb, w, radius=True)
    want = _via_plan(rb, jobs, tuning)
    got = _noalloc_c_abi(rb, jobs, tuning)
    for k in range(len(jobs)):
        assert np.array_equal(got[k], want[k]), k
    # a second call with fewer jobs and fewer fragments: the array keeps the
    # first call's tables, which must not leak into this result
    small = []
    for j in jobs[3:9]:
        n = max(1, (j["frags"].shape[0] // 3) // j["params"]["view_width"] * j["params"]["view_width"])
        small.append(dict(j, frags=j["frags"][:n].contiguous(),
                          out=torch.full((n,), 5 if j["mode"] == 0 else -2.0, dtype=j["out"].dtype, device="cuda")))
    want2 = _via_plan(rb, small, tuning)
    got2 = _noalloc_c_abi(rb, small, tuning)
    for k in range(len(small)):
        assert np.array_equal(got2[k], want2[k]), k


def test_noalloc_full_size_workload(rb):
    """The full batched workload (66.5 M fragment evaluations) in one call."""
    w = synth.make_batched(4001)
    maps, jobs = _jobs(rb, w)
    want = _via_plan(rb, jobs, (32, 1, 2048, 0, 0, 0, 4))
    got = _noalloc_c_abi(rb, jobs, (32, 1, 2048, 0, 0, 0, 4))
    for k in range(len(jobs)):
        assert np.array_equal(got[k], want[k]), k
    del maps, jobs
    torch.cuda.empty_cache()
