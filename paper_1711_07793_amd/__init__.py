"""MI355X-native revectorization-based shadow mapping (arXiv 1711.07793).

Thin Python binding of the C ABI in ``include/rbsm.h``: argument marshalling
only.  Every step of the pass runs in the HIP kernels of ``librbsm.so``;
PyTorch supplies device memory and the current stream.  There is no CPU
fallback: if the library is missing the call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librbsm.so")

RBSM_OK = 0
RBSM_ERR_INVALID_ARG = -1
RBSM_ERR_HIP = -2


class RbsmParams(ctypes.Structure):
    """Mirror of ``rbsm_params`` (include/rbsm.h)."""
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("pitch", ctypes.c_int64),
                ("depth_bias", ctypes.c_float), ("max_dist", ctypes.c_int32),
                ("kernel_radius", ctypes.c_int32), ("view_width", ctypes.c_int32)]


@dataclass
class Params:
    width: int
    height: int
    pitch: int | None = None
    depth_bias: float = 0.0
    max_dist: int = 16
    kernel_radius: int = 0
    view_width: int = 0

    def to_c(self) -> RbsmParams:
        return RbsmParams(int(self.width), int(self.height),
                          int(self.width if self.pitch is None else self.pitch),
                          float(self.depth_bias), int(self.max_dist), int(self.kernel_radius),
                          int(self.view_width))


class RbsmTuning(ctypes.Structure):
    """Mirror of ``rbsm_tuning`` (include/rbsm.h)."""
    _fields_ = [("tile_w", ctypes.c_int32), ("apron", ctypes.c_int32), ("lds_cap", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("walk_first", ctypes.c_int32), ("walk_block", ctypes.c_int32),
                ("xcd_chunk", ctypes.c_int32)]

    def __init__(self, tile_w=32, apron=1, lds_cap=2048, persistent=0, walk_first=0, walk_block=0, xcd_chunk=-1):
        super().__init__(tile_w, apron, lds_cap, persistent, walk_first, walk_block, xcd_chunk)

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class RbsmJob(ctypes.Structure):
    """Mirror of ``rbsm_job`` (include/rbsm.h)."""
    _fields_ = [("shadow_map", ctypes.c_void_p), ("frags", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("params", RbsmParams), ("mode", ctypes.c_int32), ("out", ctypes.c_void_p)]


class RbsmRequestLight(ctypes.Structure):
    """Mirror of ``rbsm_request_light``."""
    _fields_ = [("light", ctypes.c_int32), ("mode", ctypes.c_int32), ("frags", ctypes.c_void_p),
                ("depth_bias", ctypes.c_float), ("max_dist", ctypes.c_int32), ("kernel_radius", ctypes.c_int32),
                ("weight", ctypes.c_float), ("out", ctypes.c_void_p)]


class RbsmRequest(ctypes.Structure):
    """Mirror of ``rbsm_request``."""
    _fields_ = [("n", ctypes.c_int64), ("view_width", ctypes.c_int32), ("n_lights", ctypes.c_int32),
                ("lights", RbsmRequestLight * 8), ("composite", ctypes.c_void_p), ("stream", ctypes.c_void_p)]


class RbsmEngineStats(ctypes.Structure):
    """Mirror of ``rbsm_engine_stats``."""
    _fields_ = [(f, ctypes.c_int64) for f in ("submitted", "completed", "queued", "inflight", "launches",
                                              "jobs_launched", "fragments_completed", "arena_bytes",
                                              "arena_peak_bytes", "gpu_busy_ns", "inflight_bytes",
                                              "inflight_peak_bytes", "uploaded_bytes")]


class RbsmError(RuntimeError):
    pass


_lib = None


def load_library() -> ctypes.CDLL:
    """Load librbsm.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RbsmError(f"HIP library {LIB_PATH} is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    P = ctypes.POINTER(RbsmParams)
    for name in ("rbsm_visibility", "rsmss_visibility", "sm_visibility"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, i64, P, vp, vp]
        fn.restype = ctypes.c_int
    lib.rbsm_footprint.argtypes = [vp, vp, i64, P, ctypes.c_int32, vp, vp]
    lib.rbsm_footprint.restype = ctypes.c_int
    lib.rbsm_default_tuning.argtypes = []
    lib.rbsm_default_tuning.restype = RbsmTuning
    lib.rbsm_pass_tuned.argtypes = [ctypes.c_int32, vp, vp, i64, P, ctypes.POINTER(RbsmTuning), vp, vp]
    lib.rbsm_pass_tuned.restype = ctypes.c_int
    PP = ctypes.POINTER(ctypes.c_void_p)
    lib.rbsm_plan_create.argtypes = [ctypes.POINTER(RbsmJob), ctypes.c_int32, ctypes.POINTER(RbsmTuning), PP]
    lib.rbsm_plan_create.restype = ctypes.c_int
    lib.rbsm_plan_update.argtypes = [vp, ctypes.POINTER(RbsmJob), ctypes.c_int32]
    lib.rbsm_plan_update.restype = ctypes.c_int
    lib.rbsm_plan_launch.argtypes = [vp, vp]
    lib.rbsm_plan_launch.restype = ctypes.c_int
    lib.rbsm_plan_autotune.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(RbsmTuning)]
    lib.rbsm_plan_autotune.restype = ctypes.c_int
    lib.rbsm_tune_cache_load.argtypes = [ctypes.c_char_p]
    lib.rbsm_tune_cache_load.restype = ctypes.c_int
    lib.rbsm_tune_cache_save.argtypes = [ctypes.c_char_p]
    lib.rbsm_tune_cache_save.restype = ctypes.c_int
    lib.rbsm_tune_cache_clear.argtypes = []
    lib.rbsm_tune_cache_clear.restype = None
    lib.rbsm_plan_set_tuning.argtypes = [vp, ctypes.POINTER(RbsmTuning)]
    lib.rbsm_plan_set_tuning.restype = ctypes.c_int
    lib.rbsm_plan_get_tuning.argtypes = [vp, ctypes.POINTER(RbsmTuning)]
    lib.rbsm_plan_get_tuning.restype = ctypes.c_int
    lib.rbsm_plan_capture.argtypes = [vp, vp]
    lib.rbsm_plan_capture.restype = ctypes.c_int
    lib.rbsm_plan_fragments.argtypes = [vp]
    lib.rbsm_plan_fragments.restype = ctypes.c_int64
    lib.rbsm_plan_destroy.argtypes = [vp]
    lib.rbsm_plan_destroy.restype = None
    lib.rbsm_batch_launch_noalloc.argtypes = [ctypes.POINTER(RbsmJob), ctypes.c_int32, ctypes.POINTER(RbsmTuning), vp]
    lib.rbsm_batch_launch_noalloc.restype = ctypes.c_int
    d = ctypes.c_double
    lib.rbsm_rasterize.argtypes = [vp, ctypes.c_int32, d, d, d, ctypes.c_int32, ctypes.c_int32, i64, vp, vp]
    lib.rbsm_rasterize.restype = ctypes.c_int
    lib.rbsm_composite.argtypes = [i64, ctypes.c_int32, vp, vp, vp, vp, vp]
    lib.rbsm_composite.restype = ctypes.c_int
    lib.rbsm_engine_create.argtypes = [i64, ctypes.c_int32, PP]
    lib.rbsm_engine_create.restype = ctypes.c_int
    lib.rbsm_engine_add_light.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, i64, ctypes.POINTER(ctypes.c_int32)]
    lib.rbsm_engine_add_light.restype = ctypes.c_int
    lib.rbsm_engine_submit.argtypes = [vp, ctypes.POINTER(RbsmRequest), ctypes.POINTER(ctypes.c_int64)]
    lib.rbsm_engine_submit.restype = ctypes.c_int
    lib.rbsm_engine_wait.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.rbsm_engine_wait.restype = ctypes.c_int
    lib.rbsm_engine_get_stats.argtypes = [vp, ctypes.POINTER(RbsmEngineStats)]
    lib.rbsm_engine_get_stats.restype = ctypes.c_int
    lib.rbsm_engine_abort.argtypes = [vp, ctypes.c_char_p]
    lib.rbsm_engine_abort.restype = ctypes.c_int
    lib.rbsm_engine_destroy.argtypes = [vp]
    lib.rbsm_engine_destroy.restype = None
    lib.rbsm_last_error.argtypes = []
    lib.rbsm_last_error.restype = ctypes.c_char_p
    lib.rbsm_abi_version.argtypes = []
    lib.rbsm_abi_version.restype = ctypes.c_int32
    _lib = lib
    return lib


def rbsm_last_error() -> str:
    return load_library().rbsm_last_error().decode()


def rbsm_abi_version() -> int:
    return int(load_library().rbsm_abi_version())


def _params(params, shadow_map: torch.Tensor) -> RbsmParams:
    if isinstance(params, RbsmParams):
        return params
    if isinstance(params, dict):
        params = Params(**{k: v for k, v in params.items() if k in Params.__dataclass_fields__})
    p = params.to_c()
    if params.pitch is None and shadow_map.dim() == 2:
        p.pitch = shadow_map.stride(0)
    return p


def _check_inputs(shadow_map: torch.Tensor, frags: torch.Tensor):
    for name, t in (("shadow_map", shadow_map), ("frags", frags)):
        if t.device.type != "cuda":
            raise RbsmError(f"{name} must be a device tensor")
        if t.dtype != torch.float32:
            raise RbsmError(f"{name} must be float32")
    if shadow_map.dim() == 2 and shadow_map.stride(1) != 1:
        raise RbsmError("shadow_map rows must be contiguous")
    if not frags.is_contiguous() or frags.numel() % 3 != 0:
        raise RbsmError("frags must be contiguous (u, v, z) triples")


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _call(name: str, *args):
    st = getattr(load_library(), name)(*args)
    if st != RBSM_OK:
        raise RbsmError(f"{name} returned {st}: {rbsm_last_error()}")


def rbsm_visibility(shadow_map: torch.Tensor, frags: torch.Tensor, params, out: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """Hard RBSM mask (uint8 [N], 1 = lit) of ``frags`` [N, 3] against ``shadow_map`` [H, pitch]."""
    _check_inputs(shadow_map, frags)
    n = frags.numel() // 3
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=frags.device)
    p = _params(params, shadow_map)
    _call("rbsm_visibility", shadow_map.data_ptr(), frags.data_ptr(), n, ctypes.byref(p), out.data_ptr(),
          _stream(stream))
    return out


def rsmss_visibility(shadow_map: torch.Tensor, frags: torch.Tensor, params, out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
    """RSMSS visibility (float32 [N] in [0, 1]); RPCF when params.kernel_radius > 0."""
    _check_inputs(shadow_map, frags)
    n = frags.numel() // 3
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=frags.device)
    p = _params(params, shadow_map)
    _call("rsmss_visibility", shadow_map.data_ptr(), frags.data_ptr(), n, ctypes.byref(p), out.data_ptr(),
          _stream(stream))
    return out


def sm_visibility(shadow_map: torch.Tensor, frags: torch.Tensor, params, out: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """Plain shadow mapping (Eq. 1): uint8 [N], 1 = lit."""
    _check_inputs(shadow_map, frags)
    n = frags.numel() // 3
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=frags.device)
    p = _params(params, shadow_map)
    _call("sm_visibility", shadow_map.data_ptr(), frags.data_ptr(), n, ctypes.byref(p), out.data_ptr(),
          _stream(stream))
    return out


def rbsm_default_tuning() -> RbsmTuning:
    return load_library().rbsm_default_tuning()


def rbsm_pass_tuned(mode: int, shadow_map: torch.Tensor, frags: torch.Tensor, params, tuning,
                    out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Hard (mode 0) or RSMSS radius-0 (mode 1) pass under an explicit tuning
    (tile_w, apron, lds_cap); results equal the untuned entry points."""
    _check_inputs(shadow_map, frags)
    n = frags.numel() // 3
    if out is None:
        out = torch.empty(n, dtype=torch.uint8 if mode == 0 else torch.float32, device=frags.device)
    p = _params(params, shadow_map)
    t = tuning if isinstance(tuning, RbsmTuning) else RbsmTuning(*tuning)
    _call("rbsm_pass_tuned", int(mode), shadow_map.data_ptr(), frags.data_ptr(), n, ctypes.byref(p),
          ctypes.byref(t), out.data_ptr(), _stream(stream))
    return out


def rbsm_footprint(shadow_map: torch.Tensor, frags: torch.Tensor, params, mode: int,
                   touched: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Mark every texel the pass reads (uint8 [H, W]); mode 0 = hard, 1 = RSMSS."""
    _check_inputs(shadow_map, frags)
    n = frags.numel() // 3
    p = _params(params, shadow_map)
    if touched is None:
        touched = torch.zeros((p.height, p.width), dtype=torch.uint8, device=frags.device)
    _call("rbsm_footprint", shadow_map.data_ptr(), frags.data_ptr(), n, ctypes.byref(p), int(mode),
          touched.data_ptr(), _stream(stream))
    return touched


def tune_cache_load(path: str) -> int:
    """Load autotuner choices from a text file; returns the entries read."""
    lib = load_library()
    st = lib.rbsm_tune_cache_load(os.fsencode(path))
    if st < 0:
        raise RbsmError(f"rbsm_tune_cache_load returned {st}: {rbsm_last_error()}")
    return st


def tune_cache_save(path: str) -> None:
    _call("rbsm_tune_cache_save", os.fsencode(path))


def tune_cache_clear() -> None:
    load_library().rbsm_tune_cache_clear()


class Plan:
    """Batched form: one launch (or graph replay) for many (view, light) jobs.

    ``jobs`` is a list of dicts with ``map`` (float32 device tensor [H, pitch]),
    ``frags`` (float32 device tensor [N, 3]), ``params`` (dict or Params,
    kernel_radius 0, or > 0 for an RPCF job in mode 1), ``mode`` (0 hard, 1 RSMSS) and ``out`` (uint8 [N] or
    float32 [N] device tensor).  The tensors are kept alive by the plan.
    """

    def __init__(self, jobs, tuning=None):
        self._lib = load_library()
        self._h = ctypes.c_void_p()
        arr, keep = self._marshal(jobs)
        t = None if tuning is None else ctypes.byref(
            tuning if isinstance(tuning, RbsmTuning) else RbsmTuning(*tuning))
        st = self._lib.rbsm_plan_create(arr, len(jobs), t, ctypes.byref(self._h))
        if st != RBSM_OK:
            raise RbsmError(f"rbsm_plan_create returned {st}: {rbsm_last_error()}")
        self._keep = keep

    @staticmethod
    def _marshal(jobs):
        arr = (RbsmJob * len(jobs))()
        keep = []
        for k, j in enumerate(jobs):
            m, f, o = j["map"], j["frags"], j["out"]
            _check_inputs(m, f)
            mode = int(j.get("mode", 0))
            want = torch.uint8 if mode == 0 else torch.float32
            if o.dtype != want or not o.is_contiguous() or o.numel() != f.numel() // 3:
                raise RbsmError(f"job {k}: out must be a contiguous {want} tensor of N elements")
            arr[k] = RbsmJob(m.data_ptr(), f.data_ptr(), f.numel() // 3, _params(j["params"], m), mode,
                             o.data_ptr())
            keep += [m, f, o]
        return arr, keep

    def update(self, jobs):
        arr, keep = self._marshal(jobs)
        _call("rbsm_plan_update", self._h, arr, len(jobs))
        self._keep = keep

    def launch(self, stream=None):
        _call("rbsm_plan_launch", self._h, _stream(stream))

    def autotune(self, reps: int = 5, stream=None, force: bool = False) -> RbsmTuning:
        """Run the project autotuner (or apply its cached choice for this
        device and job layout unless ``force``)."""
        t = RbsmTuning()
        _call("rbsm_plan_autotune", self._h, _stream(stream), int(reps), 1 if force else 0, ctypes.byref(t))
        return t

    @property
    def tuning(self) -> RbsmTuning:
        t = RbsmTuning()
        _call("rbsm_plan_get_tuning", self._h, ctypes.byref(t))
        return t

    @tuning.setter
    def tuning(self, t):
        t = t if isinstance(t, RbsmTuning) else RbsmTuning(*t)
        _call("rbsm_plan_set_tuning", self._h, ctypes.byref(t))

    def capture(self, stream):
        _call("rbsm_plan_capture", self._h, _stream(stream))

    @property
    def fragments(self) -> int:
        return int(self._lib.rbsm_plan_fragments(self._h))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.rbsm_plan_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: ctypes may already be gone
            pass


def batch_launch_noalloc(jobs, tuning=None, stream=None) -> None:
    """One batched pass of ``jobs`` (as for ``Plan``) through the entry point
    that allocates no device memory (its tables live in a per-GPU array of the
    library).  Calls on one GPU must not overlap."""
    arr, keep = Plan._marshal(jobs)
    t = None if tuning is None else ctypes.byref(tuning if isinstance(tuning, RbsmTuning) else RbsmTuning(*tuning))
    _call("rbsm_batch_launch_noalloc", arr, len(jobs), t, _stream(stream))
    del keep


PRIM_BYTES = 112  # sizeof(rbsm_prim)


def rbsm_rasterize(prims: torch.Tensor, receiver, width: int, height: int, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """Rasterize primitives (a device uint8 tensor holding rbsm_prim records,
    e.g. ``torch.from_numpy(records.view(np.uint8)).cuda()``) over the receiver
    plane (r0, ru, rv) into a float32 [height, width] depth map (or into
    ``out``, a 2-D device tensor with contiguous rows)."""
    if prims.device.type != "cuda" or prims.dtype != torch.uint8 or not prims.is_contiguous() \
            or prims.numel() % PRIM_BYTES:
        raise RbsmError("rbsm_rasterize: prims must be contiguous device bytes of 112-byte records")
    if out is None:
        out = torch.empty((height, width), dtype=torch.float32, device=prims.device)
    if out.device.type != "cuda" or out.dtype != torch.float32 or out.dim() != 2 or out.stride(1) != 1 \
            or out.shape[0] < height or out.shape[1] < width:
        raise RbsmError("rbsm_rasterize: out must be a float32 device map with contiguous rows")
    n = prims.numel() // PRIM_BYTES
    r0, ru, rv = receiver
    _call("rbsm_rasterize", prims.data_ptr() if n else None, n, float(r0), float(ru), float(rv), int(width),
          int(height), out.stride(0), out.data_ptr(), _stream(stream))
    return out


def rbsm_composite(vis: list, modes: list, weights: list, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Weighted sum of per-light visibilities (device tensors: uint8 masks for
    mode 0, float32 for mode 1) into one float32 tensor."""
    if not 1 <= len(vis) <= 8 or len(modes) != len(vis) or len(weights) != len(vis):
        raise RbsmError("rbsm_composite: need 1..8 lights with one mode and weight each")
    n = vis[0].numel()
    for v, m in zip(vis, modes):
        if v.device.type != "cuda" or v.numel() != n or not v.is_contiguous():
            raise RbsmError("rbsm_composite: visibilities must be contiguous device tensors of one length")
        if v.dtype != (torch.uint8 if m == 0 else torch.float32):
            raise RbsmError("rbsm_composite: mode 0 needs uint8, mode 1 float32")
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=vis[0].device)
    ptrs = (ctypes.c_void_p * len(vis))(*[v.data_ptr() for v in vis])
    md = (ctypes.c_int32 * len(vis))(*modes)
    w = (ctypes.c_float * len(vis))(*weights)
    _call("rbsm_composite", n, len(vis), ptrs, md, w, out.data_ptr(), _stream(stream))
    return out


class Engine:
    """Serving engine (``rbsm_engine_*``): continuous batching of shadow
    requests over resident shadow maps, admitted by an HBM budget.

    ``submit`` takes one view: ``n`` fragments, a layout hint and 1..8
    lights, each ``dict(light=id, mode=0|1, frags=<float32 [n, 3]>,
    depth_bias=, max_dist=, kernel_radius=, weight=, out=<tensor or None>)``,
    plus an optional float32 ``composite`` tensor.  Fragments and result
    tensors on the GPU are used in place; host tensors (pinned, for overlap)
    are staged in the engine's arena.  The request's kernels wait for the
    work enqueued so far on ``stream`` (default: the current torch stream),
    which may produce its inputs asynchronously.  The tensors are kept alive
    until ``wait`` returns for that ticket.
    """

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 64):
        self._lib = load_library()
        self._h = ctypes.c_void_p()
        st = self._lib.rbsm_engine_create(int(hbm_budget_bytes), int(max_inflight), ctypes.byref(self._h))
        if st != RBSM_OK:
            raise RbsmError(rbsm_last_error())
        self._keep = {}
        self._maps = []

    def add_light(self, shadow_map: torch.Tensor) -> int:
        if shadow_map.device.type != "cuda" or shadow_map.dtype != torch.float32 or shadow_map.dim() != 2 \
                or shadow_map.stride(1) != 1:
            raise RbsmError("add_light: need a 2-D float32 device tensor with contiguous rows")
        lid = ctypes.c_int32()
        st = self._lib.rbsm_engine_add_light(self._h, shadow_map.data_ptr(), shadow_map.shape[1],
                                             shadow_map.shape[0], shadow_map.stride(0), ctypes.byref(lid))
        if st != RBSM_OK:
            raise RbsmError(rbsm_last_error())
        self._maps.append(shadow_map)
        return int(lid.value)

    def submit(self, n: int, lights: list, view_width: int = 0, composite: torch.Tensor | None = None,
               stream=None) -> int:
        q, keep = self.build_request(n, lights, view_width, composite, stream)
        return self.submit_built(q, keep)

    def abort(self, reason: str = "aborted by the caller") -> None:
        """Fail every queued and admitted request (their waits raise) once the
        work already enqueued has finished; later submissions are rejected."""
        st = self._lib.rbsm_engine_abort(self._h, reason.encode())
        if st != RBSM_OK:
            raise RbsmError(rbsm_last_error())

    def submit_built(self, q: "RbsmRequest", keep=None) -> int:
        """Submit a request built by ``build_request`` (marshalling done ahead
        of time)."""
        t = ctypes.c_int64()
        st = self._lib.rbsm_engine_submit(self._h, ctypes.byref(q), ctypes.byref(t))
        if st != RBSM_OK:
            raise RbsmError(rbsm_last_error())
        self._keep[int(t.value)] = keep
        return int(t.value)

    def build_request(self, n: int, lights: list, view_width: int = 0, composite: torch.Tensor | None = None,
                      stream=None):
        """Marshal one request into an ``RbsmRequest``; returns it with the
        tensors that must stay alive until it completes."""
        if not 1 <= len(lights) <= 8:
            raise RbsmError("submit: need 1..8 lights")
        q = RbsmRequest()
        q.n, q.view_width, q.n_lights = int(n), int(view_width), len(lights)
        q.stream = _stream(stream)
        keep = [composite]
        for i, L in enumerate(lights):
            f = L["frags"]
            if f.dtype != torch.float32 or not f.is_contiguous() or f.numel() != 3 * n:
                raise RbsmError("submit: frags must be contiguous float32 tensors of n triples")
            out = L.get("out")
            if out is not None:
                want = torch.uint8 if L.get("mode", 0) == 0 else torch.float32
                if out.dtype != want or out.numel() != n or not out.is_contiguous():
                    raise RbsmError("submit: out must be a contiguous tensor of n results of the mode's type")
            q.lights[i] = RbsmRequestLight(int(L["light"]), int(L.get("mode", 0)), f.data_ptr(),
                                           float(L.get("depth_bias", 0.0)), int(L.get("max_dist", 16)),
                                           int(L.get("kernel_radius", 0)), float(L.get("weight", 1.0)),
                                           out.data_ptr() if out is not None else None)
            keep += [f, out]
        if composite is not None:
            if composite.dtype != torch.float32 or composite.numel() != n or not composite.is_contiguous():
                raise RbsmError("submit: composite must be a contiguous float32 tensor of n values")
            q.composite = composite.data_ptr()
        return q, keep

    def wait(self, ticket: int, timeout_ms: int = -1):
        """Latency in ms (submit to results on the host), or None on time-out."""
        ms = ctypes.c_double()
        st = self._lib.rbsm_engine_wait(self._h, int(ticket), int(timeout_ms), ctypes.byref(ms))
        if st == 0:
            return None
        self._keep.pop(int(ticket), None)
        if st < 0:
            raise RbsmError(rbsm_last_error())
        return float(ms.value)

    def stats(self) -> dict:
        s = RbsmEngineStats()
        if self._lib.rbsm_engine_get_stats(self._h, ctypes.byref(s)) != RBSM_OK:
            raise RbsmError(rbsm_last_error())
        return {f: int(getattr(s, f)) for f, _ in RbsmEngineStats._fields_}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.rbsm_engine_destroy(h)
            self._h = None
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: ctypes may already be gone
            pass


__all__ = ["batch_launch_noalloc", "tune_cache_load", "tune_cache_save", "tune_cache_clear", "Engine", "rbsm_rasterize", "rbsm_composite", "RbsmRequest", "RbsmRequestLight", "RbsmEngineStats", "Plan", "RbsmJob", "Params", "RbsmParams", "RbsmTuning", "RbsmError", "rbsm_default_tuning", "rbsm_pass_tuned", "rbsm_visibility", "rsmss_visibility", "sm_visibility",
           "rbsm_footprint", "rbsm_last_error", "rbsm_abi_version", "load_library", "LIB_PATH"]
