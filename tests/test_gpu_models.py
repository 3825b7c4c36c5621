"""GPU parity of the paper's other motion models (Sec. IV-B.1 one-track model
for vehicles, Sec. IV-B.3 pedestrian acceleration model with its speed cap)
through the C ABI against the FP64 oracle: the 11-object scene on both
models, the Table I scene with one-track vehicles, low speeds (the
steady-state branch), stops and the cap, mixed with kinematic objects,
outlines, batches and the risk over time."""
import os

import numpy as np
import pytest

import oracle
from paper_2005_06773_amd import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu

THREADS = int(os.environ.get("MHC_ORACLE_THREADS", "16"))


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def mhc():
    from paper_2005_06773_amd import mhc as m
    return m


@pytest.fixture(scope="module")
def ctx(mhc):
    c = mhc.mhc_create(0)
    yield c
    mhc.mhc_destroy(c)


@pytest.mark.parametrize("seed", [10, 11, 12])
def test_models_scene_parity(mhc, ctx, seed):
    s = sg.models_scene(seed)
    say(f"11-object scene on the one-track and pedestrian acceleration models, seed {seed}")
    o = oracle.evaluate(s, threads=THREADS)
    parity.check(s, mhc.mhc_evaluate(ctx, s), o, f"models seed {seed}")
    assert (o.k64 >= 0).sum() > 500


def test_table_one_one_track_parity(mhc, ctx):
    """The Table I S1 scene with every vehicle on the one-track model: 2058
    EGO trajectories (6 accelerations on [-9.7, 9.7] x 343 steering angles)
    at 20 ms steps, the Euler step stable at speed."""
    s = sg.paper_scene(5, n_co=3)
    for o in s.objects:
        o.model = sg.MODEL_ONE_TRACK
        o.params = sg.one_track_params(o.length)
        o.u = sg.accel_grid(6, -9.7, 9.7)
        o.w = sg.steer_grid(len(o.w))
        o.score = sg.vehicle_scores(o.u, o.w)
    say("Table I S1 on the one-track model")
    o = oracle.evaluate(s, threads=THREADS)
    parity.check(s, mhc.mhc_evaluate(ctx, s), o, "Table I one-track")
    assert o.obj_crit[0] > 0.01


def _slow_scene(seed):
    """Slow one-track vehicles (both branches of the lateral update, stops)
    and accelerating pedestrians near their cap, packed together."""
    rng = np.random.default_rng(seed)
    objs = []
    for k in range(4):
        o = sg.draw_vehicle(rng, 8.0, 0.0, 7.0, 5, 7)
        o.model = sg.MODEL_ONE_TRACK
        o.params = sg.one_track_params(o.length)
        o.u = sg.accel_grid(5, -9.7, 9.7)
        o.w = sg.steer_grid(7, 0.3)
        objs.append(o)
    for k in range(3):
        o = sg.draw_pedestrian(rng, 6.0, 1.5, 3.5, 5, 6)
        o.model = sg.MODEL_PED_ACCEL
        o.params = np.array([2.7])
        o.u = sg.ped_accel_grid(5)
        o.w = sg.abs_heading_grid(6)
        o.score = None
        objs.append(o)
    objs.append(sg.draw_pedestrian(rng, 6.0, 0.0, 2.0, 4, 5))   # a kinematic pedestrian
    return sg.Scene(objs, 40, 0.1)


@pytest.mark.parametrize("seed", range(4))
def test_slow_and_capped_parity(mhc, ctx, seed):
    s = _slow_scene(300 + seed)
    say(f"slow one-track vehicles and capped pedestrians, seed {300 + seed}")
    parity.check(s, mhc.mhc_evaluate(ctx, s), oracle.evaluate(s, threads=THREADS), f"slow {seed}")


def test_models_with_outlines_timeline_and_batch(mhc, ctx):
    s = sg.models_scene(13)
    for o in s.objects:
        if o.kind == sg.VEHICLE:
            o.outline = sg.car_outline(o.length, o.width)
    s.timeline = 1
    say("models + octagons + risk over time")
    parity.check(s, mhc.mhc_evaluate(ctx, s), oracle.evaluate(s, threads=THREADS), "models octagons timeline")
    scenes = [sg.models_scene(20 + k) if k % 2 else sg.eleven_object_scene(20 + k) for k in range(6)]
    outs = mhc.mhc_evaluate_batch(ctx, scenes)
    for k, sc in enumerate(scenes):
        parity.same_results(mhc.mhc_evaluate(ctx, sc), outs[k], f"batch scene {k}")
