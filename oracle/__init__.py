"""FP64 CPU oracle for the multi-hypothesis criticality hot path.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It loads
``liboracle.so`` (built from ``mhc_oracle.c`` with gcc) and shares no code
with the GPU library; both sides are fed from the seeded generator in
``paper_2005_06773_amd.scenegen``, which holds no arithmetic of the method.

Every quantity here follows Sanchez Morales et al. (IEEE IV 2019):
probabilities Sec. IV-D.1, trajectories Sec. IV-B.1 / IV-B.3, pairs and
overlap Sec. IV-C.1, risk Sec. IV-D / IV-D.2. The readings taken where the
paper is silent are listed at the top of ``mhc_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mhc_oracle.c")
# ORACLE_LIB_PATH names another build of the same source (the sanitizer
# build of the CPU tests).
LIB = os.environ.get("ORACLE_LIB_PATH") or os.path.join(HERE, "liboracle.so")

#: tolerance band (metres) within which an FP32 evaluation may decide an
#: overlap either way; outside it first hits must agree bit for bit.
EPS = 1e-4

VEHICLE = 0
PEDESTRIAN = 1

#: overlap tests of the collision recognition (Sec. IV-C.1)
OVERLAP_EXACT = 0   # the closed shapes intersect
OVERLAP_PIP = 1     # a vertex of one polygon lies in the other, tested both ways

#: readings of the conditional-probability approximation (Sec. IV-D.2)
RISK_EXCLUSIVE = 0    # one object's trajectories exclusive, objects independent
RISK_INDEPENDENT = 1  # every trajectory combination an independent event


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP64, no fast-math, OpenMP rows)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        D = ctypes.c_double
        I = ctypes.c_int
        P = ctypes.c_void_p
        L.orc_probabilities.argtypes = [I, P, P]
        L.orc_trajectories.argtypes = [I, D, D, D, D, I, P, I, P, I, D, P, P, P]
        L.orc_trajectories_model.argtypes = [I, I, P, D, D, D, D, I, P, I, P, I, D, P, P, P]
        L.orc_margin_rect_rect.argtypes = [D] * 10
        L.orc_margin_rect_rect.restype = D
        L.orc_margin_rect_circle.argtypes = [D] * 8
        L.orc_margin_rect_circle.restype = D
        L.orc_margin_circle_circle.argtypes = [D] * 6
        L.orc_margin_circle_circle.restype = D
        L.orc_pairs.argtypes = [I, I, P, P]
        L.orc_count_trajectories.argtypes = [I, P]
        L.orc_count_trajectories.restype = ctypes.c_int64
        L.orc_count_combinations.argtypes = [I, P, I]
        L.orc_count_combinations.restype = ctypes.c_int64
        L.orc_margin_pip.argtypes = [I, P, P, I, P, P]
        L.orc_margin_pip.restype = D
        L.orc_margin_rect_rect_pip.argtypes = [D] * 10
        L.orc_margin_rect_rect_pip.restype = D
        L.orc_first_hits.argtypes = [I, I, P, P, P, P, P, P, P, P, I, P, P, P, I, P, P, D, I, P, P, P, P]
        L.orc_margin_poly_poly.argtypes = [I, P, P, I, P, P]
        L.orc_margin_poly_poly.restype = D
        L.orc_margin_poly_circle.argtypes = [I, P, P, D, D, D]
        L.orc_margin_poly_circle.restype = D
        L.orc_risk.argtypes = [I, I, P, P, I, P, P, P, P, P, P]
        L.orc_risk_timeline.argtypes = [I, I, P, P, I, I, P, P, P, P, P, P, P]
        L.orc_point_in_polygon.argtypes = [D, D, I, P, P]
        L.orc_rect_corners.argtypes = [D, D, D, D, D, P, P]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


# ---------------------------------------------------------------------------
# Elementary pieces
# ---------------------------------------------------------------------------

def probabilities(obj) -> np.ndarray:
    n = obj.n_traj
    p = np.empty(n, np.float64)
    s = None if obj.score is None else np.ascontiguousarray(obj.score, np.float64)
    _check(lib().orc_probabilities(n, _ptr(s), _ptr(p)), "probabilities")
    return p


#: motion models of an object (Sec. IV-B)
MODEL_KINEMATIC = 0   # vehicles acceleration x yaw rate, pedestrians speed x heading offset
MODEL_PED_ACCEL = 1   # pedestrians acceleration x absolute heading, speed capped (params[0] = v_max)
MODEL_ONE_TRACK = 2   # vehicles acceleration x steering angle, params (cf, cr, lf, lr, m, Iz)


def trajectories(obj, horizon: int, dt: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(x, y, psi), each [horizon][T]; slot t is the pose of step t+1."""
    T = obj.n_traj
    x = np.empty((horizon, T), np.float64)
    y = np.empty((horizon, T), np.float64)
    psi = np.empty((horizon, T), np.float64)
    u = np.ascontiguousarray(obj.u, np.float64)
    w = np.ascontiguousarray(obj.w, np.float64)
    model = int(getattr(obj, "model", MODEL_KINEMATIC))
    params = np.zeros(6, np.float64)
    if getattr(obj, "params", None) is not None:
        pp = np.asarray(obj.params, np.float64)
        params[:len(pp)] = pp
    _check(lib().orc_trajectories_model(int(obj.kind), model, _ptr(params), obj.x, obj.y, obj.heading, obj.speed,
                                        len(u), _ptr(u), len(w), _ptr(w), horizon, dt,
                                        _ptr(x), _ptr(y), _ptr(psi)), "trajectories")
    return x, y, psi


def margin_rect_rect(P, Q) -> float:
    """P, Q = (x, y, psi, L, W)."""
    return lib().orc_margin_rect_rect(*map(float, P), *map(float, Q))


def margin_rect_circle(P, Q) -> float:
    """P = (x, y, psi, L, W), Q = (x, y, r)."""
    return lib().orc_margin_rect_circle(*map(float, P), *map(float, Q))


def margin_circle_circle(P, Q) -> float:
    """P, Q = (x, y, r)."""
    return lib().orc_margin_circle_circle(*map(float, P), *map(float, Q))


def margin_pip(polyP: np.ndarray, polyQ: np.ndarray) -> float:
    """Point-in-polygon margin both ways of two polygons given as [n, 2]
    vertex arrays: the smallest signed distance of a vertex of one to the
    boundary of the other (negative inside)."""
    P = np.ascontiguousarray(polyP, np.float64)
    Q = np.ascontiguousarray(polyQ, np.float64)
    px, py = np.ascontiguousarray(P[:, 0]), np.ascontiguousarray(P[:, 1])
    qx, qy = np.ascontiguousarray(Q[:, 0]), np.ascontiguousarray(Q[:, 1])
    return lib().orc_margin_pip(len(px), _ptr(px), _ptr(py), len(qx), _ptr(qx), _ptr(qy))


#: most vertices of a vehicle outline
MAX_VERTICES = 8


def margin_poly_poly(polyP: np.ndarray, polyQ: np.ndarray) -> float:
    """Separating-axis margin of two convex CCW polygons [n, 2] (world
    coordinates): the largest gap along a unit edge normal, <= 0 iff they
    intersect."""
    P = np.ascontiguousarray(polyP, np.float64)
    Q = np.ascontiguousarray(polyQ, np.float64)
    px, py = np.ascontiguousarray(P[:, 0]), np.ascontiguousarray(P[:, 1])
    qx, qy = np.ascontiguousarray(Q[:, 0]), np.ascontiguousarray(Q[:, 1])
    return lib().orc_margin_poly_poly(len(px), _ptr(px), _ptr(py), len(qx), _ptr(qx), _ptr(qy))


def margin_poly_circle(poly: np.ndarray, c, r: float) -> float:
    P = np.ascontiguousarray(poly, np.float64)
    px, py = np.ascontiguousarray(P[:, 0]), np.ascontiguousarray(P[:, 1])
    return lib().orc_margin_poly_circle(len(px), _ptr(px), _ptr(py), float(c[0]), float(c[1]), float(r))


def margin_rect_rect_pip(P, Q) -> float:
    """P, Q = (x, y, psi, L, W)."""
    return lib().orc_margin_rect_rect_pip(*map(float, P), *map(float, Q))


def rect_corners(x, y, psi, L, W) -> np.ndarray:
    cx = np.empty(4, np.float64)
    cy = np.empty(4, np.float64)
    lib().orc_rect_corners(float(x), float(y), float(psi), float(L), float(W), _ptr(cx), _ptr(cy))
    return np.stack([cx, cy], axis=1)


def point_in_polygon(x, y, poly: np.ndarray) -> bool:
    vx = np.ascontiguousarray(poly[:, 0], np.float64)
    vy = np.ascontiguousarray(poly[:, 1], np.float64)
    return bool(lib().orc_point_in_polygon(float(x), float(y), len(vx), _ptr(vx), _ptr(vy)))


def pairs(n_objects: int, ego_only: bool) -> List[Tuple[int, int]]:
    n = lib().orc_pairs(n_objects, int(ego_only), None, None)
    a = np.empty(n, np.int32)
    b = np.empty(n, np.int32)
    lib().orc_pairs(n_objects, int(ego_only), _ptr(a), _ptr(b))
    return list(zip(a.tolist(), b.tolist()))


def count_trajectories(T: Sequence[int]) -> int:
    t = np.ascontiguousarray(T, np.int32)
    return int(lib().orc_count_trajectories(len(t), _ptr(t)))


def count_combinations(T: Sequence[int], ego_only: bool) -> int:
    t = np.ascontiguousarray(T, np.int32)
    return int(lib().orc_count_combinations(len(t), _ptr(t), int(ego_only)))


# ---------------------------------------------------------------------------
# Whole scene
# ---------------------------------------------------------------------------

@dataclass
class OracleResult:
    pair_a: np.ndarray          # [n_pairs] int32
    pair_b: np.ndarray
    pair_off: np.ndarray        # [n_pairs+1] int64 entry offsets
    T: np.ndarray               # [n_objects] int32
    p: np.ndarray               # [sum T] normalised probabilities
    k64: np.ndarray             # [entries] int32 first slot with m <= 0, else -1
    kstrict: np.ndarray         # [entries] first slot with m <= -EPS, else -1
    loose: Optional[np.ndarray]   # [entries, W] uint64 bit t: m(t) <= +EPS
    strict: Optional[np.ndarray]  # [entries, W] uint64 bit t: m(t) <= -EPS
    q: np.ndarray               # [sum T, n] from k64
    traj_crit: np.ndarray       # [sum T] from k64
    obj_crit: np.ndarray        # [n]    from k64
    traj_crit_lo: np.ndarray    # only pairs with a hit beyond the band count
    traj_crit_hi: np.ndarray    # every pair with a hit inside the band counts
    obj_crit_lo: np.ndarray
    obj_crit_hi: np.ndarray
    # time-resolved risk (scenes with ``timeline`` set), from k64
    obj_crit_t: Optional[np.ndarray] = None     # [n, H]
    traj_crit_t: Optional[np.ndarray] = None    # [sum T, H]
    obj_attrib: Optional[np.ndarray] = None     # [n, n]
    traj_attrib: Optional[np.ndarray] = None    # [sum T, n]
    # bounds over every first hit the band allows: latest (lo) and earliest (hi)
    obj_crit_t_lo: Optional[np.ndarray] = None
    obj_crit_t_hi: Optional[np.ndarray] = None
    traj_crit_t_lo: Optional[np.ndarray] = None
    traj_crit_t_hi: Optional[np.ndarray] = None


def scene_arrays(scene):
    objs = scene.objects
    kind = np.array([o.kind for o in objs], np.int32)
    length = np.array([o.length for o in objs], np.float64)
    width = np.array([o.width for o in objs], np.float64)
    radius = np.array([o.radius for o in objs], np.float64)
    T = np.array([o.n_traj for o in objs], np.int32)
    return kind, length, width, radius, T


def outline_arrays(scene):
    """Per object: vertex count (0 = no outline) and the body-frame outline
    padded to MAX_VERTICES, or (None, None, None) when no object has one."""
    outs = [getattr(o, "outline", None) for o in scene.objects]
    if all(o is None for o in outs):
        return None, None, None
    n = len(outs)
    nv = np.zeros(n, np.int32)
    ox = np.zeros((n, MAX_VERTICES), np.float64)
    oy = np.zeros((n, MAX_VERTICES), np.float64)
    for a, o in enumerate(outs):
        if o is None:
            continue
        o = np.asarray(o, np.float64)
        nv[a] = len(o)
        ox[a, :len(o)] = o[:, 0]
        oy[a, :len(o)] = o[:, 1]
    return nv, ox, oy


def evaluate(scene, pair_list: Optional[Sequence[Tuple[int, int]]] = None, eps: float = EPS,
             threads: int = 0, masks: bool = True, risk: bool = True) -> OracleResult:
    """Run the whole path on ``scene`` (a ``scenegen.Scene``).

    ``pair_list`` restricts the object pairs (the stress-scene sample); by
    default all pairs, or EGO-CO pairs when ``scene.pairs`` is the EGO mode.
    ``scene.overlap`` selects the overlap test (``OVERLAP_EXACT`` by default).
    """
    H, dt = int(scene.horizon), float(scene.dt)
    kind, length, width, radius, T = scene_arrays(scene)
    n = len(T)
    if pair_list is None:
        pair_list = pairs(n, scene.pairs == 1)
    pa = np.array([a for a, _ in pair_list], np.int32)
    pb = np.array([b for _, b in pair_list], np.int32)
    sizes = (T[pa].astype(np.int64) * T[pb].astype(np.int64)) if len(pa) else np.zeros(0, np.int64)
    poff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    entries = int(poff[-1])

    xs, ys, ps, pr = [], [], [], []
    for o in scene.objects:
        x, y, psi = trajectories(o, H, dt)
        xs.append(x.reshape(-1))
        ys.append(y.reshape(-1))
        ps.append(psi.reshape(-1))
        pr.append(probabilities(o))
    px = np.ascontiguousarray(np.concatenate(xs))
    py = np.ascontiguousarray(np.concatenate(ys))
    ppsi = np.ascontiguousarray(np.concatenate(ps))
    p = np.ascontiguousarray(np.concatenate(pr))

    W = (H + 63) // 64
    k64 = np.empty(entries, np.int32)
    kst = np.empty(entries, np.int32)
    loose = np.empty((entries, W), np.uint64) if masks else None
    strict = np.empty((entries, W), np.uint64) if masks else None
    overlap = int(getattr(scene, "overlap", OVERLAP_EXACT))
    nv, ox, oy = outline_arrays(scene)
    _check(lib().orc_first_hits(overlap, n, _ptr(kind), _ptr(length), _ptr(width), _ptr(radius),
                                _ptr(nv), _ptr(ox), _ptr(oy), _ptr(T), H,
                                _ptr(px), _ptr(py), _ptr(ppsi), len(pa), _ptr(pa), _ptr(pb),
                                float(eps), int(threads), _ptr(k64), _ptr(kst),
                                _ptr(loose), _ptr(strict)), "first_hits")
    res = OracleResult(pa, pb, poff, T, p, k64, kst, loose, strict,
                       *([None] * 7))
    if risk:
        model = int(getattr(scene, "risk", RISK_EXCLUSIVE))
        res.q, res.traj_crit, res.obj_crit = risk_from_hits(scene, pa, pb, (k64 >= 0), p, model)
        lo = kst >= 0
        kloose = first_loose_slot(loose) if masks else k64
        hi = kloose >= 0
        _, res.traj_crit_lo, res.obj_crit_lo = risk_from_hits(scene, pa, pb, lo, p, model)
        _, res.traj_crit_hi, res.obj_crit_hi = risk_from_hits(scene, pa, pb, hi, p, model)
        if getattr(scene, "timeline", 0):
            res.traj_crit_t, res.obj_crit_t, res.traj_attrib, res.obj_attrib = \
                risk_timeline(scene, pa, pb, k64, p, model)
            res.traj_crit_t_lo, res.obj_crit_t_lo, _, _ = risk_timeline(scene, pa, pb, kst, p, model)
            res.traj_crit_t_hi, res.obj_crit_t_hi, _, _ = risk_timeline(scene, pa, pb, kloose, p, model)
    return res


def first_loose_slot(loose: np.ndarray) -> np.ndarray:
    """Per entry, the first slot whose margin is <= +EPS (the earliest first
    hit an FP32 evaluation may legitimately report), or -1."""
    n, W = loose.shape
    out = np.full(n, -1, np.int32)
    for wd in range(W - 1, -1, -1):
        word = loose[:, wd]
        nz = word != 0
        if not nz.any():
            continue
        low = word[nz] & (~word[nz] + np.uint64(1))          # lowest set bit
        bit = np.round(np.log2(low.astype(np.float64))).astype(np.int32)
        out[nz] = 64 * wd + bit
    return out


def risk_from_hits(scene, pa: np.ndarray, pb: np.ndarray, hit: np.ndarray, p: np.ndarray,
                   model: int = RISK_EXCLUSIVE):
    """q [sum T, n], traj_crit [sum T], obj_crit [n] from a per-entry hit flag."""
    _, _, _, _, T = scene_arrays(scene)
    n = len(T)
    n_traj = int(T.sum())
    h = np.ascontiguousarray(hit, np.uint8)
    q = np.empty((n_traj, n), np.float64)
    tc = np.empty(n_traj, np.float64)
    oc = np.empty(n, np.float64)
    _check(lib().orc_risk(int(model), n, _ptr(T), _ptr(np.ascontiguousarray(p, np.float64)), len(pa),
                          _ptr(np.ascontiguousarray(pa, np.int32)), _ptr(np.ascontiguousarray(pb, np.int32)),
                          _ptr(h), _ptr(q), _ptr(tc), _ptr(oc)), "risk")
    return q, tc, oc


def risk_timeline(scene, pa: np.ndarray, pb: np.ndarray, k: np.ndarray, p: np.ndarray,
                  model: int = RISK_EXCLUSIVE):
    """Chronological scaling over time from per-entry first-hit slots ``k``
    (-1 = none): traj_crit_t [sum T, H], obj_crit_t [n, H], traj_attrib
    [sum T, n], obj_attrib [n, n]."""
    _, _, _, _, T = scene_arrays(scene)
    return risk_timeline_raw(T, int(scene.horizon), pa, pb, k, p, model)


def risk_timeline_raw(T, H: int, pa, pb, k, p, model: int = RISK_EXCLUSIVE):
    T = np.ascontiguousarray(T, np.int32)
    n = len(T)
    n_traj = int(T.sum())
    tct = np.empty((n_traj, H), np.float64)
    oct_ = np.empty((n, H), np.float64)
    tat = np.empty((n_traj, n), np.float64)
    oat = np.empty((n, n), np.float64)
    _check(lib().orc_risk_timeline(int(model), n, _ptr(T), _ptr(np.ascontiguousarray(p, np.float64)), int(H),
                                   len(pa), _ptr(np.ascontiguousarray(pa, np.int32)),
                                   _ptr(np.ascontiguousarray(pb, np.int32)),
                                   _ptr(np.ascontiguousarray(k, np.int32)),
                                   _ptr(tct), _ptr(oct_), _ptr(tat), _ptr(oat)), "risk_timeline")
    return tct, oct_, tat, oat


def risk_raw(T, pa, pb, hit, p, model: int = RISK_EXCLUSIVE):
    """orc_risk on explicit tables: (q, traj_crit, obj_crit)."""
    T = np.ascontiguousarray(T, np.int32)
    n = len(T)
    n_traj = int(T.sum())
    q = np.empty((n_traj, n), np.float64)
    tc = np.empty(n_traj, np.float64)
    oc = np.empty(n, np.float64)
    _check(lib().orc_risk(int(model), n, _ptr(T), _ptr(np.ascontiguousarray(p, np.float64)), len(pa),
                          _ptr(np.ascontiguousarray(pa, np.int32)), _ptr(np.ascontiguousarray(pb, np.int32)),
                          _ptr(np.ascontiguousarray(hit, np.uint8)), _ptr(q), _ptr(tc), _ptr(oc)), "risk")
    return q, tc, oc


def accepted_first_hits(k32: np.ndarray, res: OracleResult) -> np.ndarray:
    """Per entry, whether a first-hit slot computed in FP32 is acceptable:
    every slot before it is a miss beyond the band (no strict hit earlier), the
    slot itself is a hit or inside the band, and -1 only when no slot is a
    hit beyond the band. Without ambiguous slots this is bit equality with k64."""
    k32 = np.asarray(k32).astype(np.int64)
    kst = res.kstrict.astype(np.int64)
    none_ok = (k32 == -1) & (kst == -1)
    some = k32 >= 0
    no_strict_before = (kst == -1) | (kst >= k32)
    kk = np.where(some, k32, 0)
    word = kk // 64
    bit = (kk % 64).astype(np.uint64)
    lw = res.loose[np.arange(len(k32)), word]
    is_loose = ((lw >> bit) & np.uint64(1)) == np.uint64(1)
    return none_ok | (some & no_strict_before & is_loose)
