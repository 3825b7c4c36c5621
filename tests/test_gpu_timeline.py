"""GPU parity of the two risk readings and of the risk over time (through the
C ABI) against the FP64 oracle's chronological scaling.

Sizes: two-vehicle scenes over many seeds, the 11-object scene in full, a
Table I scene (2058 EGO trajectories: several risk chunks per object), ragged
scenes, batches and served frames mixing readings and time resolution, and
an approach sequence whose frames give an anticipation time.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
from paper_2005_06773_amd import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu

THREADS = int(os.environ.get("MHC_ORACLE_THREADS", "16"))
READINGS = [sg.RISK_EXCLUSIVE, sg.RISK_INDEPENDENT]


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


def with_flags(s, risk, timeline):
    s.risk = risk
    s.timeline = timeline
    return s


@pytest.mark.parametrize("risk", READINGS)
def test_two_vehicle_timeline_parity(mhc, ctx, risk):
    n = int(os.environ.get("MHC_PARITY_SEEDS", "2000")) // 4
    say(f"two-vehicle scenes, timeline, reading {risk}, seeds 0..{n - 1}")
    hits = 0
    for seed in range(n):
        s = with_flags(sg.two_vehicle_scene(seed), risk, 1)
        g = mhc.mhc_evaluate(ctx, s)
        o = oracle.evaluate(s, threads=1)
        parity.check(s, g, o, f"seed {seed}")
        hits += bool((o.k64 >= 0).any())
    assert hits > n // 50


@pytest.mark.parametrize("risk", READINGS)
@pytest.mark.parametrize("seed", [0, 1])
def test_eleven_object_timeline_parity(mhc, ctx, risk, seed):
    say(f"11-object scene seed {seed}, timeline, reading {risk}")
    s = with_flags(sg.eleven_object_scene(seed), risk, 1)
    g = mhc.mhc_evaluate(ctx, s)
    o = oracle.evaluate(s, threads=THREADS)
    parity.check(s, g, o, f"11-object seed {seed} reading {risk}")
    assert o.obj_crit.max() > 0.01


@pytest.mark.parametrize("risk", READINGS)
def test_independent_reading_without_timeline(mhc, ctx, risk):
    """The reading changes q, crit and C; the first hits stay the same."""
    s = with_flags(sg.eleven_object_scene(3), risk, 0)
    g = mhc.mhc_evaluate(ctx, s)
    parity.check(s, g, oracle.evaluate(s, threads=THREADS), f"reading {risk}")


def test_timeline_leaves_plain_results_bit_identical(mhc, ctx):
    """The per-slot sums add up to the same integers as the plain sums, so q,
    crit and C (and the first hits) are identical with and without the
    timeline, for both readings and every tile variant."""
    for risk in READINGS:
        for seed in (1, 4):
            plain = mhc.mhc_evaluate(ctx, with_flags(sg.eleven_object_scene(seed), risk, 0))
            tl = mhc.mhc_evaluate(ctx, with_flags(sg.eleven_object_scene(seed), risk, 1))
            parity.same_results(plain, {k: v for k, v in tl.items() if k not in mhc.TIMELINE_FIELDS},
                                f"reading {risk} seed {seed}")
    s = with_flags(sg.eleven_object_scene(2), sg.RISK_INDEPENDENT, 1)
    ref = None
    for v in range(mhc.MHC_N_VARIANTS):
        mhc.mhc_set_variant(ctx, v)
        got = mhc.mhc_evaluate(ctx, s)
        if ref is None:
            ref = got
        parity.same_results(ref, got, f"variant {v}")
    mhc.mhc_set_variant(ctx, -1)


@pytest.mark.parametrize("risk", READINGS)
def test_table_one_scene_timeline_parity(mhc, ctx, risk):
    """EGO of 2058 trajectories against 3 COs over 100 steps of 20 ms: the
    time-resolved kernel spans 9 chunks of the EGO, 100 slots."""
    s = with_flags(sg.paper_scene(5, n_co=3), risk, 1)
    say(f"Table I S1 scene, timeline, reading {risk}")
    g = mhc.mhc_evaluate(ctx, s)
    o = oracle.evaluate(s, threads=THREADS)
    parity.check(s, g, o, f"Table I S1 reading {risk}")
    assert o.obj_crit[0] > 0.01


def _ragged_scenes():
    out = {}
    rng = np.random.default_rng(41)
    # prime grids, pedestrians first, a horizon that is not a multiple of anything
    objs = [sg.SceneObject(sg.PEDESTRIAN, 0.5, 0.2, 0.3, 1.2, 0, 0, 0.3, sg.ped_speed_grid(3), sg.ped_heading_grid(7)),
            sg.SceneObject(sg.VEHICLE, 3.0, -1.0, 2.0, 6.0, 4.4, 1.7, 0, sg.accel_grid(5), sg.yaw_grid(11),
                           rng.uniform(0.1, 1.0, 55)),
            sg.SceneObject(sg.VEHICLE, -4.0, 2.0, -0.7, 3.0, 4.7, 1.9, 0, sg.accel_grid(13), sg.yaw_grid(1)),
            sg.SceneObject(sg.PEDESTRIAN, 1.0, 3.0, 4.0, 0.8, 0, 0, 0.3, sg.ped_speed_grid(2), sg.ped_heading_grid(3))]
    out["ragged_all_pairs"] = sg.Scene(objs, 37, 0.1)
    out["ragged_ego_pairs"] = sg.Scene([objs[1], objs[0], objs[2], objs[3]], 23, 0.1, pairs=sg.PAIRS_EGO)
    # one trajectory each, one step: the degenerate grid
    one = [sg.SceneObject(sg.VEHICLE, 0, 0, 0, 0, 4.5, 1.8, 0, np.array([0.0]), np.array([0.0])),
           sg.SceneObject(sg.VEHICLE, 2.0, 0.5, 0.4, 0, 4.5, 1.8, 0, np.array([0.0]), np.array([0.0]))]
    out["single_trajectories_H1"] = sg.Scene(one, 1, 0.1)
    # a long horizon (300 slots) with a 257 x 129 pair
    big = [sg.SceneObject(sg.VEHICLE, 0, 0, 0, 8.0, 4.5, 1.8, 0, np.linspace(-8, 3, 257), np.array([0.0])),
           sg.SceneObject(sg.VEHICLE, 60, 0.3, np.pi, 6.0, 4.5, 1.8, 0, np.linspace(-8, 3, 3), sg.yaw_grid(43))]
    out["long_horizon_257x129"] = sg.Scene(big, 300, 0.02)
    return out


@pytest.mark.parametrize("name", list(_ragged_scenes().keys()))
@pytest.mark.parametrize("risk", READINGS)
def test_ragged_timeline_parity(mhc, ctx, name, risk):
    s = with_flags(_ragged_scenes()[name], risk, 1)
    say(f"ragged timeline scene {name}, reading {risk}")
    parity.check(s, mhc.mhc_evaluate(ctx, s), oracle.evaluate(s, threads=THREADS), name)


def test_batch_mixing_readings_and_timeline(mhc, ctx):
    """A batch of scenes with every combination of reading and timeline: each
    result is bit-identical to the scene evaluated alone."""
    scenes = sg.batch_scenes(12, 16)
    for k, s in enumerate(scenes):
        with_flags(s, READINGS[k % 2], (k // 2) % 2)
    say("batch of 16 mixed scenes")
    outs = mhc.mhc_evaluate_batch(ctx, scenes)
    for k, s in enumerate(scenes):
        alone = mhc.mhc_evaluate(ctx, s)
        parity.same_results(alone, outs[k], f"batch scene {k}")
        if s.timeline:
            assert outs[k]["crit_t"] is not None and not np.isnan(outs[k]["crit_t"]).any()
    small = [k for k, s in enumerate(scenes) if s.timeline and
             sum(o.n_traj for o in s.objects) ** 2 * s.horizon < 2e8][:3]
    for k in small:
        parity.check(scenes[k], outs[k], oracle.evaluate(scenes[k], threads=THREADS), f"batch scene {k} vs oracle")


def test_plan_async_graph_and_rerun_with_timeline(mhc, ctx):
    """Plan (eager and graph replays), asynchronous evaluation into torch
    tensors, and the risk stage run again on the same sums: identical to
    mhc_evaluate."""
    import torch
    s = with_flags(sg.paper_scene(6, n_co=3), sg.RISK_INDEPENDENT, 1)
    ref = mhc.mhc_evaluate(ctx, s)
    plan = mhc.mhc_plan_create(ctx, s)
    mhc.mhc_plan_execute(plan)
    parity.same_results(ref, mhc.mhc_plan_download(plan), "plan")
    for rep in range(2):
        mhc.mhc_plan_execute_stages(plan, mhc.MHC_STAGE_RISK)
        parity.same_results(ref, mhc.mhc_plan_download(plan), f"risk stage again {rep}")
    mhc.mhc_plan_set_graph(plan, True)
    for rep in range(3):
        mhc.mhc_plan_execute(plan)
        parity.same_results(ref, mhc.mhc_plan_download(plan), f"graph replay {rep}")
        mhc.mhc_evaluate(ctx, sg.two_vehicle_scene(rep))
        torch.cuda.synchronize()
    cs = mhc.CScene(s)
    ws = torch.empty(mhc.mhc_query_sizes(cs)["device_bytes"], dtype=torch.uint8, device="cuda")
    out, r = mhc.device_result(cs)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        mhc.mhc_evaluate_async(ctx, cs, ws, r, stream)
    stream.synchronize()
    parity.same_results(ref, {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}, "async")
    out2, r2 = mhc.device_result(cs)
    mhc.mhc_plan_execute(plan, r2, stream)
    stream.synchronize()
    parity.same_results(ref, {k: (None if v is None else v.cpu().numpy()) for k, v in out2.items()}, "plan into torch")
    plan.close()


def test_timeline_outputs_need_the_flag(mhc, ctx):
    s = sg.two_vehicle_scene(3)
    cs = mhc.CScene(s)
    out, r = mhc.host_result(cs, timeline=True)
    st = mhc.lib.mhc_evaluate(ctx, ctypes.byref(cs.c), ctypes.byref(r))
    assert st == mhc.MHC_E_INVAL and "timeline" in mhc.mhc_last_error(ctx)
    assert np.all(np.isnan(out["object_crit"])) and np.all(np.isnan(out["crit_t"]))
    mhc.mhc_evaluate(ctx, s)


def test_served_timeline_frames_identical_alone(mhc, ctx):
    scenes = sg.batch_scenes(13, 12)
    for k, s in enumerate(scenes):
        with_flags(s, READINGS[k % 2], 1 if k % 3 else 0)
    alone = [mhc.mhc_evaluate(ctx, s) for s in scenes]
    srv = mhc.Server(ctx, budget=1 << 30, inflight=2)
    tickets = [srv.submit(k, s, first_hit=True, q=True) for k, s in enumerate(scenes)]
    got = [srv.wait(t)[0] for t in tickets]
    srv.stop()
    for k in range(len(scenes)):
        parity.same_results(alone[k], got[k], f"served frame {k}")
        if scenes[k].timeline:
            assert not np.isnan(got[k]["crit_t"]).any()


def test_approach_sequence_anticipation(mhc, ctx):
    """An EGO driving at a stopped vehicle, one frame every 100 ms until
    contact: all frames in one batch, each against the oracle; the
    anticipation time read from the GPU's criticality series equals the one
    read from the oracle's wherever no frame sits within the tolerance of the
    threshold."""
    frames, event = sg.approach_sequence(8)
    say(f"approach sequence: {len(frames)} frames, event at frame {event}")
    outs = mhc.mhc_evaluate_batch(ctx, frames)
    orcs = [oracle.evaluate(f, threads=THREADS) for f in frames]
    for k, (f, g, o) in enumerate(zip(frames, outs, orcs)):
        parity.check(f, g, o, f"frame {k}")
    gc = np.array([g["object_crit"][0] for g in outs])
    oc = np.array([o.obj_crit[0] for o in orcs])
    assert gc[-1] > 0.5 and gc[0] < gc[-1]
    checked = 0
    for thr in (0.1, 0.25, 0.5, 0.75, 0.9):
        if np.min(np.abs(oc - thr)) <= 1e-6:
            continue
        a_gpu = mhc.mhc_anticipation_time(gc, 0.1, thr, event)
        a_orc = mhc.mhc_anticipation_time(oc, 0.1, thr, event)
        assert a_gpu == a_orc, (thr, a_gpu, a_orc)
        say(f"  threshold {thr}: anticipation {a_gpu:.1f} s")
        checked += 1
    assert checked >= 3
