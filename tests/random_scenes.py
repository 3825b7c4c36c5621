"""Seeded random scenes that mix every scene option: object kinds and
counts, rectangles and convex outlines, the kinematic, one-track and
pedestrian-acceleration grids, scores or uniform probabilities, all pairs or
EGO pairs, exact or point-in-polygon overlap, both risk readings, the risk
over time, horizons from 1 step to several 64-step chunks (ragged ones
included) and three step lengths. Objects start close together so that
many trajectory pairs collide. Test helper: builds scenes only."""
from __future__ import annotations

import math

import numpy as np

from paper_2005_06773_amd import scenegen as sg

HORIZONS = (1, 2, 5, 30, 37, 64, 65, 100, 131)
STEPS = (0.02, 0.05, 0.1)


def _scores(rng, n: int):
    if rng.uniform() < 0.3:
        return None
    s = rng.uniform(0.0, 1.0, n)
    s[rng.uniform(0.0, 1.0, n) < 0.2] = 0.0     # some impossible trajectories
    if s.sum() == 0.0:
        s[rng.integers(n)] = 1.0
    return s


def _vehicle(rng) -> sg.SceneObject:
    length, width = float(rng.uniform(3.5, 5.5)), float(rng.uniform(1.6, 2.2))
    o = sg.SceneObject(sg.VEHICLE, float(rng.uniform(-15, 15)), float(rng.uniform(-15, 15)),
                       float(rng.uniform(0, 2 * math.pi)), float(rng.uniform(0, 15)), length=length, width=width)
    n_u, n_w = int(rng.integers(1, 10)), int(rng.integers(1, 10))
    if rng.uniform() < 0.25:
        o.model = sg.MODEL_ONE_TRACK
        o.params = sg.one_track_params(length)
        o.u = sg.accel_grid(n_u, -9.7, 9.7)
        o.w = sg.steer_grid(n_w) if n_w > 1 else np.array([0.0])
    else:
        o.u = sg.accel_grid(n_u)
        o.w = sg.yaw_grid(n_w)
    o.score = _scores(rng, n_u * n_w)
    if rng.uniform() < 0.25:
        o.outline = sg.random_convex_outline(rng, int(rng.integers(3, 9)), radius=width / 2, stretch=length / width)
    return o


def _pedestrian(rng) -> sg.SceneObject:
    o = sg.SceneObject(sg.PEDESTRIAN, float(rng.uniform(-15, 15)), float(rng.uniform(-15, 15)),
                       float(rng.uniform(0, 2 * math.pi)), float(rng.uniform(0, 2)),
                       radius=float(rng.uniform(0.25, 0.5)))
    n_u, n_w = int(rng.integers(1, 10)), int(rng.integers(1, 10))
    if rng.uniform() < 0.3:
        o.model = sg.MODEL_PED_ACCEL
        o.params = np.array([2.7])
        o.u = sg.ped_accel_grid(n_u) if n_u > 1 else np.array([0.0])
        o.w = sg.abs_heading_grid(n_w)
    else:
        o.u = sg.ped_speed_grid(n_u)
        o.w = sg.ped_heading_grid(n_w)
    o.score = _scores(rng, n_u * n_w)
    return o


def random_scene(seed: int) -> sg.Scene:
    """Scene `seed` of the sweep. The point-in-polygon test takes vehicles
    only, and EGO pairs a vehicle as object 0, as the scene rules ask."""
    rng = np.random.default_rng(70_000 + seed)
    n = int(rng.integers(2, 7))
    pip = rng.uniform() < 0.3
    ego = rng.uniform() < 0.3
    objs = []
    for k in range(n):
        vehicle = pip or (k == 0 and (ego or rng.uniform() < 0.8)) or rng.uniform() < 0.55
        objs.append(_vehicle(rng) if vehicle else _pedestrian(rng))
    s = sg.Scene(objs, int(rng.choice(HORIZONS)), float(rng.choice(STEPS)))
    s.pairs = sg.PAIRS_EGO if ego else sg.PAIRS_ALL
    s.overlap = sg.OVERLAP_PIP if pip else sg.OVERLAP_EXACT
    s.risk = sg.RISK_INDEPENDENT if rng.uniform() < 0.3 else sg.RISK_EXCLUSIVE
    s.timeline = 1 if rng.uniform() < 0.3 else 0
    return s
