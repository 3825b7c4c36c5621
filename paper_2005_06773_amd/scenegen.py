"""Seeded synthetic traffic scenes.

This module only draws inputs: initial states, control grids and trajectory
scores. It holds none of the method's arithmetic (no trajectory integration,
no overlap test, no probability), so both the GPU library's binding and the
FP64 oracle can be fed from it without sharing code.

Workloads (the paper's 20 designed scenarios and 547 recorded situations,
Sec. VI-A, are not available; these seeded scenes stand in for them):

* ``two_vehicle_scene``  2 vehicles, 5x5 grids, 30 steps of 0.1 s.
* ``eleven_object_scene`` 6 vehicles + 5 pedestrians, 15x15 grids, 30 steps.
* ``batch_scenes``       64 scenes of 3..24 objects, grid side 7..20, 20..50 steps.
* ``stress_scene``       24 vehicles + 16 pedestrians, 32x32 grids, 50 steps.
* ``paper_scene``        the execution-time experiment of Sec. VI-B (Table I):
                         EGO 6 x 343 trajectories against 3 (S1) or 10 (S2)
                         COs of 6 x 7, 100 steps of 20 ms, EGO-CO pairs only;
                         86,436,000 checks for S2.
* ``paper_shaped_sizes`` the trajectory counts of Sec. IV-B.4 / Table I.

Per object the draws happen in index order: x, y, heading, speed, then for
vehicles a length factor and a width factor. Object 0 is the EGO vehicle and
vehicles come before pedestrians.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Tuple, List, Optional

import numpy as np

VEHICLE = 0
PEDESTRIAN = 1
PAIRS_ALL = 0
PAIRS_EGO = 1
OVERLAP_EXACT = 0   # closed shapes intersect
OVERLAP_PIP = 1     # the paper's point-in-polygon test, both ways (vehicles only)
MODEL_KINEMATIC = 0   # vehicles acceleration x yaw rate, pedestrians speed x heading offset
MODEL_PED_ACCEL = 1   # pedestrians acceleration x absolute heading, speed in [0, v_max]; params = [v_max]
MODEL_ONE_TRACK = 2   # vehicles acceleration x front steering angle; params = [cf, cr, lf, lr, m, Iz]
RISK_EXCLUSIVE = 0    # one object's trajectories mutually exclusive (default)
RISK_INDEPENDENT = 1  # every trajectory combination an independent event


@dataclasses.dataclass
class SceneObject:
    kind: int
    x: float
    y: float
    heading: float
    speed: float
    length: float = 0.0   # full extent along the heading (vehicles)
    width: float = 0.0    # full extent across the heading (vehicles)
    radius: float = 0.0   # pedestrians
    u: np.ndarray = None  # vehicles: accelerations; pedestrians: speeds
    w: np.ndarray = None  # vehicles: yaw rates;     pedestrians: heading offsets
    score: Optional[np.ndarray] = None  # n_u*n_w non-negative, index k*n_w+l
    outline: Optional[np.ndarray] = None  # vehicles: [k, 2] convex CCW polygon in the body frame (3 <= k <= 8)
    model: int = 0                        # MODEL_*: motion model of the trajectory grid
    params: Optional[np.ndarray] = None   # model parameters (see MODEL_*)

    @property
    def n_traj(self) -> int:
        return int(len(self.u) * len(self.w))


@dataclasses.dataclass
class Scene:
    objects: List[SceneObject]
    horizon: int
    dt: float
    pairs: int = PAIRS_ALL
    overlap: int = OVERLAP_EXACT
    risk: int = RISK_EXCLUSIVE
    timeline: int = 0     # 1: also the criticality over time and its attribution

    @property
    def n_objects(self) -> int:
        return len(self.objects)

    def traj_counts(self) -> List[int]:
        return [o.n_traj for o in self.objects]


# --------------------------------------------------------------------------
# Control grids
# --------------------------------------------------------------------------

def accel_grid(n: int, a_min: float = -8.0, a_max: float = 3.0) -> np.ndarray:
    """Longitudinal samples following Sec. IV-B.2(a): the minimum, the maximum
    and zero, with the remaining samples equally spaced in the negative range.
    For n=5 on [-8, 3]: -8, -5.333, -2.667, 0, 3. Returned ascending."""
    if n < 1:
        raise ValueError("n must be >= 1")
    if n == 1:
        return np.array([0.0])
    if n == 2:
        return np.array([a_min, a_max])
    interior = [a_min * k / (n - 2) for k in range(n - 3, 0, -1)]
    return np.array([a_min] + interior + [0.0, a_max], dtype=np.float64)


def yaw_grid(n: int, limit: float = 0.5) -> np.ndarray:
    return np.linspace(-limit, limit, n) if n > 1 else np.array([0.0])


def ped_speed_grid(n: int, v_max: float = 2.5) -> np.ndarray:
    return np.linspace(0.0, v_max, n) if n > 1 else np.array([0.0])


def ped_heading_grid(n: int) -> np.ndarray:
    """Heading offsets 2*pi*l/n relative to the measured heading; the paper's
    0..360 degree range (Sec. IV-B.3) without the duplicated end point."""
    return np.array([2.0 * math.pi * l / n for l in range(n)], dtype=np.float64)


def _wrap(a: np.ndarray) -> np.ndarray:
    return (a + math.pi) % (2.0 * math.pi) - math.pi


def vehicle_scores(u: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Synthetic trajectory scores (the paper's weights are not published,
    Sec. IV-D.1): w_acc = w_str = 0.5, c_com = c_cou = 1, and each factor falls
    linearly from 1 to 0.1 with the magnitude of the control."""
    au = np.abs(u)
    aw = np.abs(w)
    fu = 1.0 - 0.9 * au / au.max() if au.max() > 0 else np.ones_like(u)
    fw = 1.0 - 0.9 * aw / aw.max() if aw.max() > 0 else np.ones_like(w)
    return (0.5 * fu[:, None] + 0.5 * fw[None, :]).reshape(-1).astype(np.float64)


def pedestrian_scores(s: np.ndarray, h: np.ndarray, v0: float) -> np.ndarray:
    ds = np.abs(s - v0)
    dh = np.abs(_wrap(h))
    fs = 1.0 - 0.9 * ds / ds.max() if ds.max() > 0 else np.ones_like(s)
    fh = 1.0 - 0.9 * dh / math.pi
    return (0.5 * fs[:, None] + 0.5 * fh[None, :]).reshape(-1).astype(np.float64)


# --------------------------------------------------------------------------
# Objects
# --------------------------------------------------------------------------

def draw_vehicle(rng, xy_half: float, v_lo: float, v_hi: float, n_u: int, n_w: int,
                 jitter: float = 0.1, base_len: float = 4.5, base_wid: float = 1.8) -> SceneObject:
    x = float(rng.uniform(-xy_half, xy_half))
    y = float(rng.uniform(-xy_half, xy_half))
    heading = float(rng.uniform(0.0, 2.0 * math.pi))
    speed = float(rng.uniform(v_lo, v_hi))
    lf = float(rng.uniform(1.0 - jitter, 1.0 + jitter)) if jitter > 0 else 1.0
    wf = float(rng.uniform(1.0 - jitter, 1.0 + jitter)) if jitter > 0 else 1.0
    u = accel_grid(n_u)
    w = yaw_grid(n_w)
    return SceneObject(VEHICLE, x, y, heading, speed, base_len * lf, base_wid * wf, 0.0,
                       u, w, vehicle_scores(u, w))


def draw_pedestrian(rng, xy_half: float, v_lo: float, v_hi: float, n_u: int, n_w: int,
                    radius: float = 0.3) -> SceneObject:
    x = float(rng.uniform(-xy_half, xy_half))
    y = float(rng.uniform(-xy_half, xy_half))
    heading = float(rng.uniform(0.0, 2.0 * math.pi))
    speed = float(rng.uniform(v_lo, v_hi))
    u = ped_speed_grid(n_u)
    w = ped_heading_grid(n_w)
    return SceneObject(PEDESTRIAN, x, y, heading, speed, 0.0, 0.0, radius,
                       u, w, pedestrian_scores(u, w, speed))


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def two_vehicle_scene(seed: int) -> Scene:
    """2 vehicles of 4.5 x 1.8 m, xy in U[-30,30]^2, speed U(5,15), 5x5 grids
    (accelerations on [-8,3], yaw rates on [-0.5,0.5]), 30 steps of 0.1 s."""
    rng = np.random.default_rng(seed)
    objs = [draw_vehicle(rng, 30.0, 5.0, 15.0, 5, 5, jitter=0.0) for _ in range(2)]
    return Scene(objs, 30, 0.1)


def eleven_object_scene(seed: int, horizon: int = 30) -> Scene:
    """6 vehicles (4.5 x 1.8 m +-10 %, speed U(0,20), 15x15 grids) and
    5 pedestrians (r = 0.3 m, speed U(0,2), 15 speeds x 15 headings),
    xy in U[-50,50]^2, 30 steps of 0.1 s: 83,531,250 pose-pair checks."""
    rng = np.random.default_rng(seed)
    objs = [draw_vehicle(rng, 50.0, 0.0, 20.0, 15, 15) for _ in range(6)]
    objs += [draw_pedestrian(rng, 50.0, 0.0, 2.0, 15, 15) for _ in range(5)]
    return Scene(objs, horizon, 0.1)


def _batch_scene(rng) -> Scene:
    n = int(rng.integers(3, 25))
    n_v = (6 * n + 5) // 10          # round(0.6 n); never a tie
    horizon = int(rng.integers(20, 51))
    objs = []
    for k in range(n):
        s = int(rng.integers(7, 21))
        if k < n_v:
            objs.append(draw_vehicle(rng, 50.0, 0.0, 20.0, s, s))
        else:
            objs.append(draw_pedestrian(rng, 50.0, 0.0, 2.0, s, s))
    return Scene(objs, horizon, 0.1)


def batch_scenes(seed: int = 2, n: int = 64) -> List[Scene]:
    """64 scenes from one RNG stream: object count U{3..24} with round(0.6 n)
    vehicles, per-object grid side U{7..20} (same side on both axes), horizon
    U{20..50} steps of 0.1 s, other fields as the 11-object scene."""
    rng = np.random.default_rng(seed)
    return [_batch_scene(rng) for _ in range(n)]


def serving_schedule(seed: int = 3, streams: int = 32, rate_hz: float = 10.0,
                     duration_s: float = 30.0, warmup_s: float = 2.0):
    """Arrival schedule for the serving workload: each stream is a Poisson
    process at ``rate_hz`` with a start offset U(0, 100 ms). Returns a list of
    (arrival_time_s, stream_id, scene) sorted by time; frames are drawn as in
    ``batch_scenes`` from the same RNG."""
    rng = np.random.default_rng(seed)
    events = []
    for s in range(streams):
        t = float(rng.uniform(0.0, 0.1))
        while t < warmup_s + duration_s:
            events.append((t, s))
            t += float(rng.exponential(1.0 / rate_hz))
    events.sort()
    return [(t, s, _batch_scene(rng)) for (t, s) in events]


def stress_scene(seed: int = 4) -> Scene:
    """24 vehicles + 16 pedestrians, 32x32 grids (1024 trajectories each),
    50 steps of 0.1 s, xy in U[-100,100]^2: 40,894,464,000 checks."""
    rng = np.random.default_rng(seed)
    objs = [draw_vehicle(rng, 100.0, 0.0, 20.0, 32, 32) for _ in range(24)]
    objs += [draw_pedestrian(rng, 100.0, 0.0, 2.0, 32, 32) for _ in range(16)]
    return Scene(objs, 50, 0.1)


def stress_sample_pairs(n_objects: int = 40, k: int = 20, seed: int = 1004):
    """The seeded sample of object pairs the oracle checks on the stress scene."""
    pairs = [(a, b) for a in range(n_objects) for b in range(a + 1, n_objects)]
    idx = np.random.default_rng(seed).choice(len(pairs), k, replace=False)
    return [pairs[i] for i in sorted(idx)]


def paper_scene(seed: int = 5, n_co: int = 10, n_acc: int = 6, overlap: int = OVERLAP_EXACT) -> Scene:
    """The execution-time experiment of Sec. VI-B (Table I) as a seeded scene.

    The EGO drives east at U(12, 16) m/s with n_acc accelerations on [-8, 3]
    and 343 yaw rates on [-0.5, 0.5] rad/s (the paper's 7^3 paths);
    every CO (4.5 x 1.8 m +-10 %) has n_acc accelerations and 7 yaw rates.
    COs take four roles in turn: lead vehicle in the EGO's lane
    (x U(8, 40), speed U(0, 12)), oncoming in the next lane (x U(10, 60),
    y 3.5, speed U(8, 16)), crossing towards the EGO's lane (x U(15, 35),
    |y| U(8, 25), speed U(5, 12)), following (x U(-25, -8), speed U(10, 18));
    lateral jitter U(-0.5, 0.5) m, heading jitter U(-0.05, 0.05) rad.
    100 steps of 20 ms, EGO-CO pairs only: 2058 x 42 x 100 = 8,643,600
    checks per CO (86,436,000 for S2 = 10 COs, 25,930,800 for S1 = 3)."""
    rng = np.random.default_rng(seed)
    u = accel_grid(n_acc)
    w_ego = yaw_grid(343)
    ego = SceneObject(VEHICLE, 0.0, 0.0, 0.0, float(rng.uniform(12.0, 16.0)), 4.5, 1.8, 0.0,
                      u, w_ego, vehicle_scores(u, w_ego))
    objs = [ego]
    w_co = yaw_grid(7)
    for k in range(n_co):
        role = k % 4
        if role == 0:
            x, y, h, v = rng.uniform(8.0, 40.0), 0.0, 0.0, rng.uniform(0.0, 12.0)
        elif role == 1:
            x, y, h, v = rng.uniform(10.0, 60.0), 3.5, math.pi, rng.uniform(8.0, 16.0)
        elif role == 2:
            side = 1.0 if rng.uniform() < 0.5 else -1.0
            x, y, h, v = rng.uniform(15.0, 35.0), side * rng.uniform(8.0, 25.0), -side * math.pi / 2, rng.uniform(5.0, 12.0)
        else:
            x, y, h, v = rng.uniform(-25.0, -8.0), 0.0, 0.0, rng.uniform(10.0, 18.0)
        y += rng.uniform(-0.5, 0.5)
        h += rng.uniform(-0.05, 0.05)
        lf, wf = rng.uniform(0.9, 1.1), rng.uniform(0.9, 1.1)
        objs.append(SceneObject(VEHICLE, float(x), float(y), float(h), float(v), 4.5 * lf, 1.8 * wf, 0.0,
                                u, w_co, vehicle_scores(u, w_co)))
    return Scene(objs, 100, 0.02, pairs=PAIRS_EGO, overlap=overlap)


def ped_accel_grid(n: int, a_max: float = 12.0) -> np.ndarray:
    """Pedestrian accelerations equally distributed on [-a_max, a_max]
    (Sec. IV-B.3: -12 to 12 m/s^2)."""
    return np.linspace(-a_max, a_max, n)


def abs_heading_grid(n: int) -> np.ndarray:
    """Absolute headings equally distributed on [0, 2 pi), no duplicated end
    point (Sec. IV-B.3: 0 to 360 degrees)."""
    return 2.0 * math.pi * np.arange(n) / n


def steer_grid(n: int, delta_max: float = 0.1) -> np.ndarray:
    """Front steering angles on [-delta_max, delta_max] rad."""
    return np.linspace(-delta_max, delta_max, n)


# Assumed one-track parameters (the paper takes its values from handbooks it
# cites, without printing them): by length, a small, a mid-size and a large
# car; cornering stiffness per axle in N/rad, lf / lr from the centre of
# gravity to the axles, mass, yaw inertia. All understeer (lr cr > lf cf).
ONE_TRACK_CLASSES = (
    (4.0, np.array([50_000.0, 55_000.0, 1.00, 1.35, 1100.0, 1500.0])),
    (4.7, np.array([67_500.0, 75_000.0, 1.20, 1.50, 1500.0, 2500.0])),
    (1e9, np.array([90_000.0, 100_000.0, 1.35, 1.65, 2000.0, 3800.0])),
)


def one_track_params(length: float) -> np.ndarray:
    for max_len, p in ONE_TRACK_CLASSES:
        if length < max_len:
            return p.copy()
    return ONE_TRACK_CLASSES[-1][1].copy()


def models_scene(seed: int = 10, horizon: int = 30, dt: float = 0.1) -> Scene:
    """The 11-object scene on the paper's other motion models: vehicles on
    the one-track model (15 accelerations on [-9.7, 9.7] by the paper's rule
    x 15 steering angles on [-0.1, 0.1] rad, parameters by length), the
    pedestrians on the acceleration model (15 accelerations on [-12, 12] x 15
    absolute headings, speed capped at 2.7 m/s)."""
    s = eleven_object_scene(seed, horizon)
    s.dt = dt
    for o in s.objects:
        if o.kind == VEHICLE:
            o.model = MODEL_ONE_TRACK
            o.params = one_track_params(o.length)
            o.u = accel_grid(15, -9.7, 9.7)
            o.w = steer_grid(15)
            o.score = vehicle_scores(o.u, o.w)
        else:
            o.model = MODEL_PED_ACCEL
            o.params = np.array([2.7])
            o.u = ped_accel_grid(15)
            o.w = abs_heading_grid(15)
            o.score = None
    return s


def car_outline(length: float, width: float, chamfer: float = 0.35) -> np.ndarray:
    """Octagonal footprint of a car: the length x width rectangle (centred on
    the pose, x along the heading) with its corners cut by `chamfer` metres
    along both sides, counter-clockwise."""
    l, w, c = length / 2.0, width / 2.0, chamfer
    return np.array([[l, -w + c], [l, w - c], [l - c, w], [-l + c, w],
                     [-l, w - c], [-l, -w + c], [-l + c, -w], [l - c, -w]], np.float64)


def random_convex_outline(rng, k: int, radius: float = 2.0, stretch: float = 2.0) -> np.ndarray:
    """A random strictly convex polygon of k vertices, counter-clockwise,
    around the origin: k sorted angles with gaps in [0.5, 1.5] x 2 pi / k on
    an ellipse of semi-axes radius*stretch x radius, drawn again until every
    interior angle is at least 45 degrees."""
    while True:
        gaps = rng.uniform(0.5, 1.5, k)
        ang = np.cumsum(gaps) / gaps.sum() * 2 * math.pi + rng.uniform(0, 2 * math.pi)
        pts = np.stack([radius * stretch * np.cos(ang), radius * np.sin(ang)], axis=1)
        pts = pts - pts.mean(axis=0) * rng.uniform(0.0, 0.5)
        if outline_ok(pts):
            return pts


def outline_ok(poly: np.ndarray, min_angle_deg: float = 45.0) -> bool:
    """Strictly convex, counter-clockwise, interior angles >= min_angle_deg."""
    k = len(poly)
    for e in range(k):
        a, b, c = poly[e - 1], poly[e], poly[(e + 1) % k]
        u, v = a - b, c - b
        if (b[0] - a[0]) * (c[1] - b[1]) - (b[1] - a[1]) * (c[0] - b[0]) <= 0:
            return False
        cosang = np.dot(u, v) / (np.linalg.norm(u) * np.linalg.norm(v))
        if math.degrees(math.acos(max(-1.0, min(1.0, cosang)))) < min_angle_deg:
            return False
    return True


def polygon_scene(seed: int = 9, horizon: int = 30) -> Scene:
    """The 11-object scene with every vehicle given the octagonal outline of a
    car (corners chamfered 0.35 m): vehicle-vehicle pairs become polygon
    pairs (8 x 8 edges) and vehicle-pedestrian pairs polygon-circle pairs."""
    s = eleven_object_scene(seed, horizon)
    for o in s.objects:
        if o.kind == VEHICLE:
            o.outline = car_outline(o.length, o.width)
    return s


def approach_sequence(seed: int = 8, frame_dt: float = 0.1, horizon: int = 30, dt: float = 0.1,
                      side: int = 9) -> Tuple[List[Scene], int]:
    """An EGO vehicle driving at constant speed U(12, 18) m/s straight at a
    stopped vehicle U(35, 55) m ahead in its lane (lateral offset U(-0.3, 0.3)
    m), observed every frame_dt seconds as it would be if it never reacted:
    frame f has the EGO f * frame_dt * v0 further on. Both have side x side
    grids (accelerations by the paper's rule on [-8, 3], yaw rates on
    [-0.5, 0.5]); the two vehicles are 4.5 x 1.8 m +-10 %. Returns the frames
    up to (not including) the event frame, the first at which the two
    rectangles touch, and that frame index. The stand-in for the designed
    scenarios with static objects ahead of the EGO (Sec. VI-A), whose
    geometry is not published."""
    rng = np.random.default_rng(seed)
    v0 = float(rng.uniform(12.0, 18.0))
    D = float(rng.uniform(35.0, 55.0))
    y_co = float(rng.uniform(-0.3, 0.3))
    L0, W0 = 4.5 * rng.uniform(0.9, 1.1), 1.8 * rng.uniform(0.9, 1.1)
    L1, W1 = 4.5 * rng.uniform(0.9, 1.1), 1.8 * rng.uniform(0.9, 1.1)
    u, w = accel_grid(side), yaw_grid(side)
    gap = D - (L0 + L1) / 2.0
    event = int(math.ceil(gap / (v0 * frame_dt)))
    frames = []
    for f in range(event):
        ego = SceneObject(VEHICLE, v0 * f * frame_dt, 0.0, 0.0, v0, L0, W0, 0.0, u, w, vehicle_scores(u, w))
        co = SceneObject(VEHICLE, D, y_co, 0.0, 0.0, L1, W1, 0.0, u, w, vehicle_scores(u, w))
        frames.append(Scene([ego, co], horizon, dt, timeline=1))
    return frames, event


def paper_shaped_sizes(n_co: int, n_acc: int = 6, ego_paths: int = 343, co_paths: int = 7):
    """Trajectory counts of the paper's execution-time experiment (Sec. IV-B.4,
    Sec. VI-B): EGO = n_acc * 7^3, each CO = n_acc * 7."""
    return [n_acc * ego_paths] + [n_acc * co_paths] * n_co


def uniform_scores(scene: Scene) -> Scene:
    """Same scene with score arrays dropped (uniform probabilities)."""
    objs = [dataclasses.replace(o, score=None) for o in scene.objects]
    return dataclasses.replace(scene, objects=objs)
