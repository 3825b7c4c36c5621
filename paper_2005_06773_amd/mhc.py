"""ctypes binding of ``libmhc.so`` (argument marshalling only).

Every function here has the name of the C entry point it wraps (declared in
``include/mhc.h``) and does no arithmetic of the method: the whole path runs
in the library's HIP kernels. Importing this module loads the library and
fails loudly when it has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MHC_LIB_PATH names another build of the same library (the host-side
# sanitizer builds of the CPU tests); there is never a fallback.
LIB_PATH = os.environ.get("MHC_LIB_PATH") or os.path.join(HERE, "libmhc.so")

MHC_OK = 0
MHC_E_INVAL = -1
MHC_E_NOMEM = -2
MHC_E_DEVICE = -3
MHC_E_BUSY = -4
MHC_E_TIMEOUT = -5
MHC_OVERLAP_EXACT = 0
MHC_OVERLAP_PIP = 1
MHC_RISK_EXCLUSIVE = 0
MHC_RISK_INDEPENDENT = 1
_STATUS = {0: "MHC_OK", -1: "MHC_E_INVAL", -2: "MHC_E_NOMEM", -3: "MHC_E_DEVICE",
           -4: "MHC_E_BUSY", -5: "MHC_E_TIMEOUT"}

EXPORTED = [
    "mhc_create", "mhc_destroy", "mhc_last_error", "mhc_query_sizes", "mhc_anticipation_time",
    "mhc_evaluate", "mhc_evaluate_async", "mhc_evaluate_noalloc",
    "mhc_plan_create", "mhc_plan_update", "mhc_plan_execute", "mhc_plan_execute_stages", "mhc_plan_set_graph",
    "mhc_plan_download", "mhc_plan_destroy",
    "mhc_set_variant", "mhc_autotune", "mhc_autotune_batch", "mhc_tune_save", "mhc_tune_load", "mhc_plan_check",
    "mhc_evaluate_batch",
    "mhc_server_start", "mhc_server_start_executor", "mhc_submit", "mhc_wait", "mhc_server_stats",
    "mhc_server_stop",
]


class MhcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


# ---------------------------------------------------------------------------
# Structures (mirror include/mhc.h)
# ---------------------------------------------------------------------------
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)


MHC_MAX_VERTICES = 8


class mhc_object(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("x", _D), ("y", _D), ("heading", _D), ("speed", _D),
                ("length", _D), ("width", _D), ("radius", _D),
                ("n_u", ctypes.c_int32), ("n_w", ctypes.c_int32),
                ("u", _DP), ("w", _DP), ("score", _DP),
                ("n_vertices", ctypes.c_int32), ("vertices", _DP),
                ("model", ctypes.c_int32), ("params", ctypes.c_double * 6)]


class mhc_scene(ctypes.Structure):
    _fields_ = [("n_objects", ctypes.c_int32), ("objects", ctypes.POINTER(mhc_object)),
                ("horizon", ctypes.c_int32), ("dt", _D), ("pairs", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("risk", ctypes.c_int32), ("timeline", ctypes.c_int32)]


class mhc_sizes(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("n_traj_pairs", ctypes.c_int64),
                ("n_checks", ctypes.c_int64), ("device_bytes", ctypes.c_size_t)]


class mhc_plan_info(ctypes.Structure):
    _fields_ = [("n_units", ctypes.c_int64), ("n_waves", ctypes.c_int64), ("blocked_pairs", ctypes.c_int64),
                ("uncovered", ctypes.c_int64), ("repeated", ctypes.c_int64), ("out_of_range", ctypes.c_int64),
                ("contiguous", ctypes.c_int32), ("time_split", ctypes.c_int32)]


RESULT_FIELDS = ("object_crit", "traj_crit", "traj_prob", "q", "first_hit",
                 "crit_t", "traj_crit_t", "attrib", "traj_attrib")
TIMELINE_FIELDS = ("crit_t", "traj_crit_t", "attrib", "traj_attrib")


class mhc_result(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in RESULT_FIELDS]


class mhc_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_inflight_ticks", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("max_frames_per_tick", ctypes.c_int32),
                ("max_checks_per_tick", ctypes.c_int64), ("watchdog_us", ctypes.c_int64),
                ("deadline_us", ctypes.c_int64)]


class mhc_timing(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_int64), ("admit_ns", ctypes.c_int64), ("launch_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("tick", ctypes.c_int64)]


class mhc_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("deferred", ctypes.c_int64), ("ticks", ctypes.c_int64), ("checks", ctypes.c_int64),
                ("late", ctypes.c_int64),
                ("p50_ms", _D), ("p99_ms", _D), ("max_ms", _D), ("mean_ms", _D), ("checks_per_s", _D)]


#: mhc_executor callbacks: launch(user, slot, tick, n_frames, scenes, dsts), poll(user, slot)
EXECUTOR_LAUNCH = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                   ctypes.POINTER(mhc_scene), ctypes.POINTER(mhc_result))
EXECUTOR_POLL = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32)


class mhc_executor(ctypes.Structure):
    _fields_ = [("user", ctypes.c_void_p), ("launch", EXECUTOR_LAUNCH), ("poll", EXECUTOR_POLL)]


def _load():
    # One HIP runtime per process: torch ships its own copy of libamdhip64.so.7.
    # Loading torch first makes this library bind to that same copy, so device
    # pointers and streams created by torch are valid here.
    # (MHC_NO_TORCH=1: a process that never touches a GPU, such as the CPU
    # tests under a sanitizer, does without)
    if os.environ.get("MHC_NO_TORCH") != "1":
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    V = ctypes.c_void_p
    I = ctypes.c_int
    S = ctypes.c_size_t
    for name, args in {
        "mhc_create": [I, S, ctypes.POINTER(V)],
        "mhc_destroy": [V],
        "mhc_last_error": [V],
        "mhc_query_sizes": [ctypes.POINTER(mhc_scene), ctypes.POINTER(mhc_sizes)],
        "mhc_anticipation_time": [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
        "mhc_evaluate": [V, ctypes.POINTER(mhc_scene), ctypes.POINTER(mhc_result)],
        "mhc_evaluate_async": [V, ctypes.POINTER(mhc_scene), V, S, ctypes.POINTER(mhc_result), V],
        "mhc_evaluate_noalloc": [V, ctypes.POINTER(mhc_scene), ctypes.POINTER(mhc_result), V],
        "mhc_plan_create": [V, ctypes.POINTER(mhc_scene), ctypes.POINTER(V)],
        "mhc_plan_update": [V, ctypes.POINTER(mhc_scene)],
        "mhc_plan_execute": [V, ctypes.POINTER(mhc_result), V],
        "mhc_plan_execute_stages": [V, ctypes.POINTER(mhc_result), V, ctypes.c_uint32],
        "mhc_plan_set_graph": [V, ctypes.c_int32],
        "mhc_plan_download": [V, ctypes.POINTER(mhc_result)],
        "mhc_plan_destroy": [V],
        "mhc_set_variant": [V, ctypes.c_int32],
        "mhc_autotune": [V, ctypes.POINTER(mhc_scene), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_double)],
        "mhc_autotune_batch": [V, ctypes.c_int32, ctypes.POINTER(mhc_scene), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)],
        "mhc_tune_save": [V, ctypes.c_char_p],
        "mhc_tune_load": [V, ctypes.c_char_p],
        "mhc_plan_check": [ctypes.c_int32, ctypes.POINTER(mhc_scene), ctypes.c_int32, ctypes.c_int32,
                           ctypes.POINTER(mhc_plan_info)],
        "mhc_evaluate_batch": [V, ctypes.c_int32, ctypes.POINTER(mhc_scene), ctypes.POINTER(mhc_result)],
        "mhc_server_start": [V, ctypes.POINTER(mhc_server_cfg), ctypes.POINTER(V)],
        "mhc_server_start_executor": [ctypes.POINTER(mhc_server_cfg), ctypes.POINTER(mhc_executor), ctypes.POINTER(V)],
        "mhc_submit": [V, ctypes.c_int32, ctypes.POINTER(mhc_scene), ctypes.POINTER(mhc_result),
                       ctypes.POINTER(ctypes.c_uint64)],
        "mhc_wait": [V, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(mhc_timing)],
        "mhc_server_stats": [V, ctypes.POINTER(mhc_stats)],
        "mhc_server_stop": [V],
    }.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = None if name in ("mhc_destroy", "mhc_plan_destroy") else ctypes.c_int
    L.mhc_last_error.restype = ctypes.c_char_p
    return L


lib = _load()


# ---------------------------------------------------------------------------
# Marshalling
# ---------------------------------------------------------------------------

class CScene:
    """A scene (``scenegen.Scene`` or anything with the same fields) held as
    C structures; keeps its arrays alive."""

    def __init__(self, scene):
        self.keep = []
        objs = (mhc_object * scene.n_objects)()
        for k, o in enumerate(scene.objects):
            u = np.ascontiguousarray(o.u, np.float64)
            w = np.ascontiguousarray(o.w, np.float64)
            sc = None if o.score is None else np.ascontiguousarray(o.score, np.float64)
            self.keep += [u, w, sc]
            objs[k].kind = int(o.kind)
            objs[k].x, objs[k].y, objs[k].heading, objs[k].speed = float(o.x), float(o.y), float(o.heading), float(o.speed)
            objs[k].length, objs[k].width, objs[k].radius = float(o.length), float(o.width), float(o.radius)
            objs[k].n_u, objs[k].n_w = len(u), len(w)
            objs[k].u = u.ctypes.data_as(_DP)
            objs[k].w = w.ctypes.data_as(_DP)
            objs[k].score = sc.ctypes.data_as(_DP) if sc is not None else None
            objs[k].model = int(getattr(o, "model", 0))
            prm = getattr(o, "params", None)
            if prm is not None:
                for j, val in enumerate(np.asarray(prm, np.float64).reshape(-1)[:6]):
                    objs[k].params[j] = float(val)
            outline = getattr(o, "outline", None)
            if outline is not None:
                ov = np.ascontiguousarray(np.asarray(outline, np.float64).reshape(-1))
                self.keep.append(ov)
                objs[k].n_vertices = len(ov) // 2
                objs[k].vertices = ov.ctypes.data_as(_DP)
        self.objs = objs
        self.c = mhc_scene(scene.n_objects, objs, int(scene.horizon), float(scene.dt), int(scene.pairs),
                           int(getattr(scene, "overlap", MHC_OVERLAP_EXACT)),
                           int(getattr(scene, "risk", MHC_RISK_EXCLUSIVE)), int(getattr(scene, "timeline", 0)))
        self.H = int(scene.horizon)
        self.timeline = bool(getattr(scene, "timeline", 0))
        self.T = [len(o.u) * len(o.w) for o in scene.objects]
        self.n = scene.n_objects
        self.pairs = [(a, b) for a in range(self.n) for b in range(a + 1, self.n)
                      if scene.pairs == 0 or a == 0]
        self.n_traj = sum(self.T)
        self.n_hits = sum(self.T[a] * self.T[b] for a, b in self.pairs)


def _check(ctx, st: int):
    if st != MHC_OK:
        msg = lib.mhc_last_error(ctx).decode() if ctx else ""
        raise MhcError(st, msg)


def _shapes(cs: CScene, first_hit: bool, q: bool, timeline: Optional[bool]):
    tl = cs.timeline if timeline is None else timeline
    return {
        "object_crit": (cs.n,), "traj_crit": (cs.n_traj,), "traj_prob": (cs.n_traj,),
        "q": (cs.n_traj, cs.n) if q else None,
        "first_hit": (cs.n_hits,) if first_hit else None,
        "crit_t": (cs.n, cs.H) if tl else None,
        "traj_crit_t": (cs.n_traj, cs.H) if tl else None,
        "attrib": (cs.n, cs.n) if tl else None,
        "traj_attrib": (cs.n_traj, cs.n) if tl else None,
    }


def host_results(css: Sequence[CScene], first_hit: bool = True, q: bool = True,
                 timeline: Optional[bool] = None):
    """NaN-filled host outputs (first hits -2) for every field asked for, per
    scene; the time-resolved ones by default when a scene asks for the risk
    over time. Each field of all scenes is one array and each scene's output a
    view of it, and the result structs are one array of pointers, so a batch
    costs a few allocations rather than several per scene."""
    shapes = [_shapes(c, first_hit, q, timeline) for c in css]
    ptrs = np.zeros((len(css), len(RESULT_FIELDS)), np.uint64)
    outs = [dict.fromkeys(sh) for sh in shapes]
    for f, k in enumerate(RESULT_FIELDS):
        sizes = [0 if sh[k] is None else math.prod(sh[k]) for sh in shapes]
        if not any(sh[k] is not None for sh in shapes):
            continue
        buf = np.full(sum(sizes), -2, np.int16) if k == "first_hit" else np.full(sum(sizes), np.nan)
        base = buf.__array_interface__["data"][0]
        off = 0
        for i, sh in enumerate(shapes):
            if sh[k] is not None:
                outs[i][k] = buf[off:off + sizes[i]].reshape(sh[k])
                ptrs[i, f] = base + off * buf.itemsize
                off += sizes[i]
    return outs, (mhc_result * len(css)).from_buffer(ptrs)


def host_result(cs: CScene, first_hit: bool = True, q: bool = True, timeline: Optional[bool] = None):
    """``host_results`` of one scene (its outputs and its result struct), with
    an array per field."""
    out = {k: None if sh is None else (np.full(sh, -2, np.int16) if k == "first_hit" else np.full(sh, np.nan))
           for k, sh in _shapes(cs, first_hit, q, timeline).items()}
    r = mhc_result(*(None if out[k] is None else out[k].ctypes.data for k in RESULT_FIELDS))
    return out, r


# ---------------------------------------------------------------------------
# Entry points
# ---------------------------------------------------------------------------

def mhc_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = ctypes.c_void_p()
    st = lib.mhc_create(device, hbm_budget_bytes, ctypes.byref(h))
    if st != MHC_OK:
        raise MhcError(st, f"mhc_create(device={device}) failed")
    return h


def mhc_destroy(ctx):
    lib.mhc_destroy(ctx)


def mhc_last_error(ctx) -> str:
    return lib.mhc_last_error(ctx).decode()


def mhc_plan_check(scenes, variant: int, max_waves: int = 0):
    """(status, info dict) of the host-side walk of the collision plan for
    ``scenes`` (a scene or a list) with tile variant ``variant`` and
    ``max_waves`` resident waves (0: one wave per unit). No GPU needed."""
    if not isinstance(scenes, (list, tuple)):
        scenes = [scenes]
    cs = [s if isinstance(s, CScene) else CScene(s) for s in scenes]
    arr = (mhc_scene * len(cs))(*[c.c for c in cs])
    info = mhc_plan_info()
    st = lib.mhc_plan_check(len(cs), arr, variant, max_waves, ctypes.byref(info))
    return st, {k: getattr(info, k) for k, _ in mhc_plan_info._fields_}


def mhc_query_sizes(scene) -> dict:
    cs = scene if isinstance(scene, CScene) else CScene(scene)
    s = mhc_sizes()
    st = lib.mhc_query_sizes(ctypes.byref(cs.c), ctypes.byref(s))
    if st != MHC_OK:
        raise MhcError(st, "mhc_query_sizes: invalid scene")
    return {k: getattr(s, k) for k, _ in mhc_sizes._fields_}


def mhc_anticipation_time(crit: Sequence[float], frame_dt: float, threshold: float, event_frame: int) -> float:
    c = np.ascontiguousarray(crit, np.float64)
    out = ctypes.c_double()
    st = lib.mhc_anticipation_time(len(c), c.ctypes.data_as(_DP), float(frame_dt), float(threshold),
                                   int(event_frame), ctypes.byref(out))
    if st != MHC_OK:
        raise MhcError(st, "mhc_anticipation_time: invalid arguments")
    return out.value


def mhc_evaluate(ctx, scene, first_hit: bool = True, q: bool = True, timeline: Optional[bool] = None) -> dict:
    cs = scene if isinstance(scene, CScene) else CScene(scene)
    out, r = host_result(cs, first_hit, q, timeline)
    _check(ctx, lib.mhc_evaluate(ctx, ctypes.byref(cs.c), ctypes.byref(r)))
    return out


def mhc_evaluate_batch(ctx, scenes: Sequence, first_hit: bool = True, q: bool = True) -> List[dict]:
    css = [s if isinstance(s, CScene) else CScene(s) for s in scenes]
    arr = (mhc_scene * len(css))(*[c.c for c in css])
    outs, rarr = host_results(css, first_hit, q)
    _check(ctx, lib.mhc_evaluate_batch(ctx, len(css), arr, rarr))
    return outs


def device_result(cs: CScene, device="cuda", first_hit: bool = True, q: bool = True,
                  timeline: Optional[bool] = None):
    """Torch-owned device outputs for the asynchronous and plan paths."""
    import torch
    out = {}
    for k, sh in _shapes(cs, first_hit, q, timeline).items():
        if sh is None:
            out[k] = None
        elif k == "first_hit":
            out[k] = torch.full(sh, -2, dtype=torch.int16, device=device)
        else:
            out[k] = torch.full(sh, float("nan"), dtype=torch.float64, device=device)
    r = mhc_result(*(None if out[k] is None else out[k].data_ptr() for k in RESULT_FIELDS))
    return out, r


def mhc_evaluate_async(ctx, scene, workspace, dev_out: mhc_result, stream=None):
    """``workspace``: a torch uint8 CUDA tensor of >= device_bytes bytes;
    ``stream``: a torch.cuda.Stream (default: the current stream)."""
    import torch
    cs = scene if isinstance(scene, CScene) else CScene(scene)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(ctx, lib.mhc_evaluate_async(ctx, ctypes.byref(cs.c), workspace.data_ptr(), workspace.numel(),
                                       ctypes.byref(dev_out), ctypes.c_void_p(s.cuda_stream)))
    return cs


MHC_NOALLOC_MAX_BYTES = 64 << 20


def mhc_evaluate_noalloc(ctx, scene, dev_out: mhc_result, stream=None):
    """Like ``mhc_evaluate_async`` with the library's own device array as the
    workspace; ``stream``: a torch.cuda.Stream (default: the current stream)."""
    import torch
    cs = scene if isinstance(scene, CScene) else CScene(scene)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(ctx, lib.mhc_evaluate_noalloc(ctx, ctypes.byref(cs.c), ctypes.byref(dev_out),
                                         ctypes.c_void_p(s.cuda_stream)))
    return cs


class Plan:
    def __init__(self, ctx, scene):
        self.ctx = ctx
        self.cs = scene if isinstance(scene, CScene) else CScene(scene)
        self.h = ctypes.c_void_p()
        _check(ctx, lib.mhc_plan_create(ctx, ctypes.byref(self.cs.c), ctypes.byref(self.h)))

    def close(self):
        if self.h:
            lib.mhc_plan_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mhc_plan_create(ctx, scene) -> Plan:
    return Plan(ctx, scene)


def mhc_plan_update(plan: Plan, scene):
    cs = scene if isinstance(scene, CScene) else CScene(scene)
    _check(plan.ctx, lib.mhc_plan_update(plan.h, ctypes.byref(cs.c)))
    plan.cs = cs


def mhc_plan_execute(plan: Plan, dev_out: Optional[mhc_result] = None, stream=None):
    sp = 0 if stream is None else (stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    _check(plan.ctx, lib.mhc_plan_execute(plan.h, ctypes.byref(dev_out) if dev_out is not None else None,
                                          ctypes.c_void_p(sp)))


MHC_STAGE_TRAJ, MHC_STAGE_COLLIDE, MHC_STAGE_RISK, MHC_STAGE_ALL = 1, 2, 4, 7


def mhc_plan_execute_stages(plan: Plan, stages: int, dev_out: Optional[mhc_result] = None, stream=None):
    sp = 0 if stream is None else (stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    _check(plan.ctx, lib.mhc_plan_execute_stages(plan.h, ctypes.byref(dev_out) if dev_out is not None else None,
                                                 ctypes.c_void_p(sp), stages))


def mhc_plan_set_graph(plan: Plan, enable: bool):
    _check(plan.ctx, lib.mhc_plan_set_graph(plan.h, int(bool(enable))))


def mhc_plan_download(plan: Plan, first_hit: bool = True, q: bool = True) -> dict:
    out, r = host_result(plan.cs, first_hit, q)
    _check(plan.ctx, lib.mhc_plan_download(plan.h, ctypes.byref(r)))
    return out


def mhc_plan_destroy(plan: Plan):
    plan.close()


# ---- tile autotuning -------------------------------------------------------

MHC_N_VARIANTS = 4


def mhc_set_variant(ctx, variant: int):
    _check(ctx, lib.mhc_set_variant(ctx, variant))


def mhc_autotune(ctx, scene, reps: int = 20):
    """Returns (best variant, [microseconds per launch of each variant])."""
    cs = scene if isinstance(scene, CScene) else CScene(scene)
    best = ctypes.c_int32()
    us = (ctypes.c_double * MHC_N_VARIANTS)()
    _check(ctx, lib.mhc_autotune(ctx, ctypes.byref(cs.c), reps, ctypes.byref(best), us))
    return best.value, list(us)


def mhc_autotune_batch(ctx, scenes: Sequence, reps: int = 10):
    """Tunes the variant of batches like ``scenes`` (one collision launch for
    all); returns (best variant, [microseconds per launch of each variant])."""
    css = [s if isinstance(s, CScene) else CScene(s) for s in scenes]
    arr = (mhc_scene * len(css))(*[c.c for c in css])
    best = ctypes.c_int32()
    us = (ctypes.c_double * MHC_N_VARIANTS)()
    _check(ctx, lib.mhc_autotune_batch(ctx, len(css), arr, reps, ctypes.byref(best), us))
    return best.value, list(us)


def mhc_tune_save(ctx, path: str):
    _check(ctx, lib.mhc_tune_save(ctx, path.encode()))


def mhc_tune_load(ctx, path: str):
    _check(ctx, lib.mhc_tune_load(ctx, path.encode()))


# ---- server ---------------------------------------------------------------

class Server:
    """A server on the GPU of ``ctx`` (mhc_server_start), or, with ``ctx``
    None and ``executor`` = (launch, poll) Python callables, on that executor
    (mhc_server_start_executor): launch(slot, tick, n, scenes, dsts) -> status,
    poll(slot) -> 1 done / 0 running / < 0 failed."""

    def __init__(self, ctx, budget: int = 0, inflight: int = 0, queue: int = 0, frames_per_tick: int = 0,
                 checks_per_tick: int = 0, watchdog_us: int = 0, deadline_us: int = 0, executor=None):
        self.ctx = ctx
        cfg = mhc_server_cfg(budget, inflight, queue, frames_per_tick, checks_per_tick, watchdog_us, deadline_us)
        self.h = ctypes.c_void_p()
        if executor is None:
            _check(ctx, lib.mhc_server_start(ctx, ctypes.byref(cfg), ctypes.byref(self.h)))
        else:
            launch, poll = executor
            self._cb = (EXECUTOR_LAUNCH(lambda user, slot, tick, n, scenes, dsts: launch(slot, tick, n, scenes, dsts)),
                        EXECUTOR_POLL(lambda user, slot: poll(slot)))
            self._ex = mhc_executor(None, *self._cb)
            st = lib.mhc_server_start_executor(ctypes.byref(cfg), ctypes.byref(self._ex), ctypes.byref(self.h))
            if st != MHC_OK:
                raise MhcError(st, "mhc_server_start_executor")
        self.pending = {}

    def submit(self, stream_id: int, scene, first_hit: bool = False, q: bool = False):
        cs = scene if isinstance(scene, CScene) else CScene(scene)
        out, r = host_result(cs, first_hit, q)
        t = ctypes.c_uint64()
        st = lib.mhc_submit(self.h, stream_id, ctypes.byref(cs.c), ctypes.byref(r), ctypes.byref(t))
        if st != MHC_OK:
            raise MhcError(st, mhc_last_error(self.ctx) if self.ctx else "mhc_submit")
        self.pending[t.value] = (out, r)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1):
        tm = mhc_timing()
        st = lib.mhc_wait(self.h, ticket, timeout_us, ctypes.byref(tm))
        if st != MHC_OK:
            if st != MHC_E_TIMEOUT:
                self.pending.pop(ticket, None)
            raise MhcError(st, "mhc_wait")
        out, _ = self.pending.pop(ticket)
        return out, {k: getattr(tm, k) for k, _ in mhc_timing._fields_}

    def stats(self) -> dict:
        s = mhc_stats()
        st = lib.mhc_server_stats(self.h, ctypes.byref(s))
        if st != MHC_OK:
            raise MhcError(st, "mhc_server_stats")
        return {k: getattr(s, k) for k, _ in mhc_stats._fields_}

    def stop(self):
        if self.h:
            h, self.h = self.h, ctypes.c_void_p()
            st = lib.mhc_server_stop(h)
            if st != MHC_OK:
                raise MhcError(st, mhc_last_error(self.ctx) if self.ctx else "mhc_server_stop")


def mhc_server_start(ctx, **kw) -> Server:
    return Server(ctx, **kw)
