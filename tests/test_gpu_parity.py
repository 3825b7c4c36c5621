"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Sizes: the 2-vehicle scene over many seeds, the 11-object scene (the size
the benchmark times) in full, ragged and degenerate shapes, the Table I
workload (86.4 M checks) in both overlap modes, point-in-polygon edge cases,
a seeded sample of 20 object pairs of the 40-object stress scene, and grids cut
into 2-D blocks of items (with and without time splits).
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2005_06773_amd import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu


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


THREADS = int(os.environ.get("MHC_ORACLE_THREADS", "16"))


def veh(x, y, psi, v, u, w, L=4.5, W=1.8, score=None):
    return sg.SceneObject(sg.VEHICLE, x, y, psi, v, L, W, 0.0, np.asarray(u, float), np.asarray(w, float), score)


def ped(x, y, psi, v, u, w, r=0.3, score=None):
    return sg.SceneObject(sg.PEDESTRIAN, x, y, psi, v, 0.0, 0.0, r, np.asarray(u, float), np.asarray(w, float), score)


TWO_VEHICLE_SEEDS = int(os.environ.get("MHC_PARITY_SEEDS", "10000"))


@pytest.mark.parametrize("chunk", range(5))
def test_two_vehicle_scene_parity(mhc, ctx, chunk):
    """The two-vehicle scene over seeds 0..9999, in five chunks."""
    per = (TWO_VEHICLE_SEEDS + 4) // 5
    seeds = range(chunk * per, min(TWO_VEHICLE_SEEDS, (chunk + 1) * per))
    say(f"two-vehicle scene, seeds {seeds.start}..{seeds.stop - 1}")
    with_hits = 0
    exact = []
    for seed in seeds:
        s = sg.two_vehicle_scene(seed)
        g = mhc.mhc_evaluate(ctx, s)
        o = oracle.evaluate(s, threads=1)
        exact.append(parity.check(s, g, o, f"seed {seed}"))
        with_hits += bool((o.k64 >= 0).any())
    say(f"  seeds with a collision: {with_hits}/{len(seeds)}; mean exact first-hit fraction {np.mean(exact):.6f}; "
        f"largest criticality deviation {parity.max_dev.get('traj_crit', 0.0):.2e}")
    assert with_hits > len(seeds) // 50


@pytest.mark.parametrize("chunk", range(10))
def test_eleven_object_scene_parity(mhc, ctx, chunk):
    """The 11-object scene (the benchmark's size and launch path) in full over
    seeds 0..99, ten seeds per test."""
    band = 0
    for seed in range(10 * chunk, 10 * chunk + 10):
        say(f"11-object scene seed {seed}")
        s = sg.eleven_object_scene(seed)
        g = mhc.mhc_evaluate(ctx, s)
        o = oracle.evaluate(s, threads=THREADS)
        ex = parity.check(s, g, o, f"seed {seed}")
        nb = int(np.sum(o.kstrict != oracle.first_loose_slot(o.loose)))
        band += nb
        say(f"  exact first-hit fraction {ex:.7f}, hits {(o.k64 >= 0).sum()}, band entries {nb}")
    say(f"  band entries in the chunk {band}; largest deviations "
        + ", ".join(f"{k} {v:.2e}" for k, v in sorted(parity.max_dev.items())))


def test_scene_far_from_the_origin(mhc, ctx):
    """Positions are taken relative to a per-scene origin before the FP32
    tests, so a scene 5-7 km from (0, 0) keeps the accuracy of one near it:
    the 11-object scene shifted by (5000.3, -7000.7) m against the oracle on
    the shifted (absolute) coordinates."""
    for seed in (1, 3):
        s = sg.eleven_object_scene(seed)
        for o in s.objects:
            o.x += 5000.3
            o.y -= 7000.7
        say(f"11-object scene seed {seed} shifted by (5000.3, -7000.7) m")
        g = mhc.mhc_evaluate(ctx, s)
        o = oracle.evaluate(s, threads=THREADS)
        ex = parity.check(s, g, o, f"shifted seed {seed}")
        say(f"  exact first-hit fraction {ex:.7f}, hits {(o.k64 >= 0).sum()}")


def _edge_scenes():
    rng = np.random.default_rng(77)
    out = {}
    out["single_trajectories_H1"] = sg.Scene([veh(0, 0, 0, 5, [0.0], [0.0]), veh(3, 0.5, 0.3, 2, [1.0], [0.1])], 1, 0.1)
    out["all_classes_ragged"] = sg.Scene([
        veh(0, 0, 0.2, 8, sg.accel_grid(7), sg.yaw_grid(11)),
        ped(6, 1, 3.0, 1.0, sg.ped_speed_grid(13), sg.ped_heading_grid(1)),
        veh(10, -2, 2.5, 6, sg.accel_grid(1), sg.yaw_grid(17)),
        ped(4, 4, 1.0, 1.5, sg.ped_speed_grid(3), sg.ped_heading_grid(19)),
    ], 37, 0.1)
    out["pedestrian_first"] = sg.Scene([
        ped(0, 0, 0.0, 1.0, sg.ped_speed_grid(5), sg.ped_heading_grid(9)),
        veh(3, 0, 3.1, 5, sg.accel_grid(5), sg.yaw_grid(5)),
        ped(1, 2, 1.0, 1.0, sg.ped_speed_grid(4), sg.ped_heading_grid(4)),
    ], 30, 0.1)
    out["overlap_at_start"] = sg.Scene([veh(0, 0, 0, 0, sg.accel_grid(5), sg.yaw_grid(5)),
                                        veh(1, 0, 0.5, 0, sg.accel_grid(5), sg.yaw_grid(5)),
                                        ped(0.5, 0.2, 0, 0, sg.ped_speed_grid(4), sg.ped_heading_grid(4))], 10, 0.1)
    out["far_apart"] = sg.Scene([veh(0, 0, 0, 5, sg.accel_grid(5), sg.yaw_grid(5)),
                                 veh(500, 500, 0, 5, sg.accel_grid(5), sg.yaw_grid(5))], 30, 0.1)
    out["tile_spanning_257x129"] = sg.Scene([veh(0, 0, 0.0, 10, sg.accel_grid(257), sg.yaw_grid(1)),
                                             veh(25, 1, math.pi, 10, sg.accel_grid(3), sg.yaw_grid(43))], 40, 0.1)
    out["long_horizon"] = sg.Scene([veh(0, 0, 0.0, 3, sg.accel_grid(4), sg.yaw_grid(3)),
                                    ped(30, 0.5, math.pi, 1.0, sg.ped_speed_grid(3), sg.ped_heading_grid(5)),
                                    veh(60, 0, math.pi, 4, sg.accel_grid(3), sg.yaw_grid(3))], 300, 0.1)
    sc = sg.eleven_object_scene(5)
    sc.objects = sc.objects[:4] + sc.objects[6:9]
    for o in sc.objects:
        o.score = None
    out["uniform_scores"] = sc
    sz = sg.eleven_object_scene(6)
    sz.objects = sz.objects[:3] + sz.objects[6:8]
    for o in sz.objects:
        o.score = o.score * (rng.uniform(size=o.score.shape) > 0.5)
        o.score[0] += 1.0
    out["zero_scores"] = sz
    se = sg.eleven_object_scene(9)
    se.pairs = sg.PAIRS_EGO
    out["ego_mode"] = se
    # the paper's EGO-only pair set at its step length, with a dense jam of COs
    jam = [veh(0, 0, 0.0, 12, sg.accel_grid(6), sg.yaw_grid(7))]
    for k in range(4):
        jam.append(veh(15 + 9 * k, 3.5 * ((k % 2) * 2 - 1) * 0.5, math.pi * (k % 2), 8, sg.accel_grid(6), sg.yaw_grid(7)))
    out["ego_jam_20ms"] = sg.Scene(jam, 100, 0.02, pairs=sg.PAIRS_EGO)
    return out


@pytest.mark.parametrize("name", list(_edge_scenes().keys()))
def test_edge_scene_parity(mhc, ctx, name):
    s = _edge_scenes()[name]
    say(f"edge scene {name}")
    g = mhc.mhc_evaluate(ctx, s)
    o = oracle.evaluate(s, threads=THREADS)
    parity.check(s, g, o, name)
    if name == "overlap_at_start":
        assert np.all(g["first_hit"] == 0)
    if name == "far_apart":
        assert np.all(g["first_hit"] == -1) and np.all(g["object_crit"] == 0)


def _pip_scenes():
    rng = np.random.default_rng(91)
    out = {}
    out["plus_sign_crossing"] = sg.Scene([veh(-10, 0, 0.0, 10, [0.0], [0.0]), veh(0, 0, math.pi / 2, 0, [0.0], [0.0])],
                                         2, 1.0, overlap=sg.OVERLAP_PIP)
    out["t_bone_20ms"] = sg.Scene([veh(-10, 0, 0.0, 10, sg.accel_grid(5), sg.yaw_grid(9)),
                                   veh(0, 0, math.pi / 2, 0, sg.accel_grid(3), sg.yaw_grid(3))], 60, 0.02,
                                  overlap=sg.OVERLAP_PIP)
    out["containment_at_start"] = sg.Scene([veh(0, 0, 0.3, 0, sg.accel_grid(5), sg.yaw_grid(5), L=8.0, W=3.0),
                                            veh(0.5, 0.2, 1.0, 0, sg.accel_grid(4), sg.yaw_grid(4), L=1.0, W=0.8)],
                                           10, 0.1, overlap=sg.OVERLAP_PIP)
    out["tile_spanning_257x129"] = sg.Scene([veh(0, 0, 0.0, 10, sg.accel_grid(257), sg.yaw_grid(1)),
                                             veh(25, 1, math.pi, 10, sg.accel_grid(3), sg.yaw_grid(43))], 40, 0.1,
                                            overlap=sg.OVERLAP_PIP)
    objs = [veh(rng.uniform(-15, 15), rng.uniform(-15, 15), rng.uniform(0, 2 * math.pi), rng.uniform(0, 12),
                sg.accel_grid(int(rng.integers(3, 9))), sg.yaw_grid(int(rng.integers(3, 12))),
                L=rng.uniform(3, 6), W=rng.uniform(1.5, 2.2)) for _ in range(6)]
    out["six_vehicles_all_pairs_coarse"] = sg.Scene(objs, 30, 0.1, overlap=sg.OVERLAP_PIP)
    return out


@pytest.mark.parametrize("name", list(_pip_scenes().keys()))
def test_pip_scene_parity(mhc, ctx, name):
    s = _pip_scenes()[name]
    say(f"point-in-polygon scene {name}")
    g = mhc.mhc_evaluate(ctx, s)
    o = oracle.evaluate(s, threads=THREADS)
    parity.check(s, g, o, name)
    if name == "plus_sign_crossing":
        assert g["first_hit"].tolist() == [-1]
        s.overlap = sg.OVERLAP_EXACT
        assert mhc.mhc_evaluate(ctx, s)["first_hit"].tolist() == [0]
    if name == "containment_at_start":
        assert np.all(g["first_hit"] == 0)


@pytest.mark.parametrize("overlap", [0, 1], ids=["exact", "pip"])
def test_table_one_workload_parity(mhc, ctx, overlap):
    """The execution-time experiment of Sec. VI-B (S2: EGO 2058 trajectories
    against 10 COs of 42, 100 steps of 20 ms, 86,436,000 checks) in full."""
    for seed in (5, 6):
        s = sg.paper_scene(seed, overlap=overlap)
        say(f"Table I S2 scene seed {seed}, overlap mode {overlap}")
        g = mhc.mhc_evaluate(ctx, s)
        o = oracle.evaluate(s, threads=THREADS)
        ex = parity.check(s, g, o, f"S2 seed {seed} overlap {overlap}")
        say(f"  exact first-hit fraction {ex:.7f}, hits {(o.k64 >= 0).sum()}")


def test_batch_mixes_overlap_modes(mhc, ctx):
    scenes = [sg.paper_scene(7, n_co=3, overlap=sg.OVERLAP_PIP), sg.eleven_object_scene(3),
              sg.paper_scene(8, n_co=3), _pip_scenes()["six_vehicles_all_pairs_coarse"]]
    outs = mhc.mhc_evaluate_batch(ctx, scenes)
    for k, (s, g) in enumerate(zip(scenes, outs)):
        parity.same_results(mhc.mhc_evaluate(ctx, s), g, f"batch scene {k}")
    parity.check(scenes[0], outs[0], oracle.evaluate(scenes[0], threads=THREADS), "batch PIP scene")


def test_every_tile_variant_is_identical(mhc, ctx):
    """Each compiled micro-tile shape and wave cut gives bit-identical results
    (first hits, q, criticality) on scenes that cover all classes and ragged
    tiles, and the first of them agrees with the oracle."""
    edge = _edge_scenes()
    scenes = {"eleven_object_seed2": sg.eleven_object_scene(2),
              "all_classes_ragged": edge["all_classes_ragged"],
              "tile_spanning_257x129": edge["tile_spanning_257x129"],
              "pip_six_vehicles": _pip_scenes()["six_vehicles_all_pairs_coarse"],
              "pip_tile_spanning": _pip_scenes()["tile_spanning_257x129"]}
    try:
        for name, s in scenes.items():
            ref = None
            for v in range(mhc.MHC_N_VARIANTS):
                say(f"variant {v}: {name}")
                mhc.mhc_set_variant(ctx, v)
                g = mhc.mhc_evaluate(ctx, s)
                if ref is None:
                    parity.check(s, g, oracle.evaluate(s, threads=THREADS), f"{name} variant {v}")
                    ref = g
                else:
                    parity.same_results(ref, g, f"{name} variant {v}")
    finally:
        mhc.mhc_set_variant(ctx, -1)


def test_plan_and_async_match_evaluate(mhc, ctx):
    import torch
    s = sg.eleven_object_scene(1)
    say("plan / async / evaluate on the 11-object scene")
    ref = mhc.mhc_evaluate(ctx, s)
    # without the first-hit output the criticality is bit for bit the same
    noh = mhc.mhc_evaluate(ctx, s, first_hit=False)
    parity.same_results({k: v for k, v in ref.items() if k != "first_hit"}, noh, "no first-hit output")
    plan = mhc.mhc_plan_create(ctx, s)
    for rep in range(3):
        mhc.mhc_plan_execute(plan)
        got = mhc.mhc_plan_download(plan)
        parity.same_results(ref, got, f"plan rep {rep}")
    # device outputs on a torch stream
    cs = mhc.CScene(s)
    sizes = mhc.mhc_query_sizes(cs)
    ws = torch.empty(sizes["device_bytes"], dtype=torch.uint8, device="cuda")
    out, r = mhc.device_result(cs)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        mhc.mhc_evaluate_async(ctx, cs, ws, r, stream)
        mhc.mhc_plan_execute(plan, r, stream)
    stream.synchronize()
    got = {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}
    parity.same_results(ref, got, "async+plan into torch tensors")
    # a plan updated with new values of the same shape equals a fresh evaluation
    s2 = sg.eleven_object_scene(2)
    mhc.mhc_plan_update(plan, s2)
    mhc.mhc_plan_execute(plan)
    parity.same_results(mhc.mhc_evaluate(ctx, s2), mhc.mhc_plan_download(plan), "plan update")
    plan.close()


def test_plans_on_concurrent_streams(mhc, ctx):
    """Steps of three plans (different scenes, each with its own workspace and
    outputs) issued round-robin on three streams overlap on the GPU; every
    plan's results equal the scene evaluated alone, after each pass."""
    import torch
    scenes = [sg.eleven_object_scene(1), sg.eleven_object_scene(2), sg.paper_scene(5, n_co=3)]
    say("three plans on three streams, 4 passes")
    refs = [mhc.mhc_evaluate(ctx, s) for s in scenes]
    plans = [mhc.mhc_plan_create(ctx, s) for s in scenes]
    outs = [mhc.device_result(mhc.CScene(s)) for s in scenes]
    streams = [torch.cuda.Stream() for _ in scenes]
    try:
        for rnd in range(4):
            for _ in range(3):
                for k in range(len(scenes)):
                    mhc.mhc_plan_execute(plans[k], outs[k][1], streams[k])
            torch.cuda.synchronize()
            for k, (o, _) in enumerate(outs):
                got = {key: (None if v is None else v.cpu().numpy()) for key, v in o.items()}
                parity.same_results(refs[k], got, f"plan {k}, pass {rnd}")
    finally:
        for pl in plans:
            pl.close()


@pytest.fixture(scope="module")
def batch64(mhc, ctx):
    """The 64-scene batch workload evaluated in one batched call."""
    scenes = sg.batch_scenes(2, 64)
    say(f"batch of {len(scenes)} scenes")
    return scenes, mhc.mhc_evaluate_batch(ctx, scenes)


def test_batch_matches_single(mhc, ctx, batch64):
    """Every scene of the batch bit for bit equal to the scene alone."""
    scenes, outs = batch64
    for k, s in enumerate(scenes):
        parity.same_results(outs[k], mhc.mhc_evaluate(ctx, s), f"batch scene {k}")


@pytest.mark.parametrize("chunk", range(4))
def test_batch_matches_oracle(mhc, ctx, batch64, chunk):
    """Every scene of the batch against the oracle, 16 scenes per test."""
    scenes, outs = batch64
    for k in range(16 * chunk, 16 * chunk + 16):
        s = scenes[k]
        say(f"batch scene {k} vs oracle ({s.n_objects} objects, horizon {s.horizon})")
        parity.check(s, outs[k], oracle.evaluate(s, threads=THREADS), f"batch scene {k} vs oracle")


def test_invalid_scenes_rejected_without_writes(mhc, ctx):
    base = sg.two_vehicle_scene(0)
    bads = []
    s = sg.two_vehicle_scene(0); s.objects[0].x = float("nan"); bads.append(s)
    s = sg.two_vehicle_scene(0); s.objects[1].length = -1.0; bads.append(s)
    s = sg.two_vehicle_scene(0); s.horizon = 0; bads.append(s)
    s = sg.two_vehicle_scene(0); s.dt = 0.0; bads.append(s)
    s = sg.two_vehicle_scene(0); s.objects[1].score = np.zeros(25); bads.append(s)
    s = sg.two_vehicle_scene(0); s.objects = s.objects[:1]; bads.append(s)
    for k, s in enumerate(bads):
        cs = mhc.CScene(s)
        out, r = mhc.host_result(cs)
        import ctypes
        st = mhc.lib.mhc_evaluate(ctx, ctypes.byref(cs.c), ctypes.byref(r))
        assert st == mhc.MHC_E_INVAL, k
        assert np.all(np.isnan(out["object_crit"])) and np.all(out["first_hit"] == -2)
        assert mhc.mhc_last_error(ctx)
    mhc.mhc_evaluate(ctx, base)  # the context still works


def test_stress_scene_sampled_pairs(mhc, ctx):
    """Full 40-object scene (40.9e9 checks) on the GPU; the oracle checks the
    seeded sample of 20 object pairs element by element."""
    s = sg.stress_scene(4)
    say("stress scene: GPU full run")
    g = mhc.mhc_evaluate(ctx, s, q=False)
    sample = sg.stress_sample_pairs(s.n_objects, 20, 1004)
    say(f"stress scene: oracle on sampled pairs {sample}")
    o = oracle.evaluate(s, pair_list=sample, threads=THREADS, risk=False)
    T = s.traj_counts()
    all_pairs = [(a, b) for a in range(s.n_objects) for b in range(a + 1, s.n_objects)]
    off = np.concatenate([[0], np.cumsum([T[a] * T[b] for a, b in all_pairs])])
    k32 = np.concatenate([g["first_hit"][off[all_pairs.index(p)]:off[all_pairs.index(p) + 1]] for p in sample])
    acc = oracle.accepted_first_hits(k32, o)
    assert acc.all(), f"{(~acc).sum()} rejected"
    say(f"  sampled entries {k32.size}, exact {np.mean(k32 == o.k64):.7f}, hits {(o.k64 >= 0).sum()}")
    assert np.all((g["object_crit"] >= 0) & (g["object_crit"] <= 1 + 1e-12))


def test_risk_stage_reruns_on_many_chunk_objects(mhc, ctx):
    """The EGO of the Table I scene has 2058 trajectories: the risk kernel
    sums its criticality over 9 chunks with a completion counter. Running
    the risk stage again on the same sums, and replaying the whole plan from
    a graph, must give the same results."""
    import torch
    s = sg.paper_scene(6, n_co=3)
    plan = mhc.mhc_plan_create(ctx, s)
    mhc.mhc_plan_execute_stages(plan, mhc.MHC_STAGE_ALL)
    first = mhc.mhc_plan_download(plan)
    parity.check(s, first, oracle.evaluate(s, threads=THREADS), "Table I S1 plan")
    for rep in range(3):
        mhc.mhc_plan_execute_stages(plan, mhc.MHC_STAGE_RISK)
        parity.same_results(first, mhc.mhc_plan_download(plan), f"risk stage again {rep}")
    mhc.mhc_plan_set_graph(plan, True)
    for rep in range(4):
        mhc.mhc_plan_execute(plan)
        parity.same_results(first, mhc.mhc_plan_download(plan), f"graph replay {rep}")
        mhc.mhc_evaluate(ctx, sg.two_vehicle_scene(rep))
        torch.cuda.synchronize()
    plan.close()


def test_graph_replays_match_eager(mhc, ctx):
    """Plans and mhc_evaluate replay captured HIP graphs. Every replay, with
    eager work and synchronisations in between, must equal the eager launch
    sequence; same-shape scenes with new values reuse a graph and must still
    match the oracle."""
    import torch
    s = sg.eleven_object_scene(4)
    plan = mhc.mhc_plan_create(ctx, s)
    mhc.mhc_plan_set_graph(plan, True)
    mhc.mhc_plan_execute_stages(plan, mhc.MHC_STAGE_ALL)     # eager
    eager = mhc.mhc_plan_download(plan)
    other = sg.two_vehicle_scene(11)
    for rep in range(5):
        mhc.mhc_plan_execute(plan)                            # graph replay
        got = mhc.mhc_plan_download(plan)
        parity.same_results(eager, got, f"plan graph replay {rep}")
        mhc.mhc_evaluate(ctx, other)                          # unrelated eager work in between
        torch.cuda.synchronize()
    plan.close()
    say("graph replays of mhc_evaluate over same-shape scenes with new values")
    for seed in (20, 21, 22):
        sc = sg.eleven_object_scene(seed)
        g = mhc.mhc_evaluate(ctx, sc)
        ref_plan = mhc.mhc_plan_create(ctx, sc)
        mhc.mhc_plan_execute_stages(ref_plan, mhc.MHC_STAGE_ALL)
        parity.same_results(mhc.mhc_plan_download(ref_plan), g, f"evaluate graph seed {seed}")
        ref_plan.close()
    sc = sg.eleven_object_scene(23)
    parity.check(sc, mhc.mhc_evaluate(ctx, sc), oracle.evaluate(sc, threads=THREADS), "evaluate graph vs oracle")
    # a shape change between calls is a different graph
    small = sg.two_vehicle_scene(5)
    parity.check(small, mhc.mhc_evaluate(ctx, small), oracle.evaluate(small), "shape change")


def _block_scenes():
    """Scenes whose item grids have sides that are multiples of 8, so the plan
    cuts them into 2-D blocks of items; short horizons leave few units for the
    resident waves, so the blocks also run with time splits."""
    rng = np.random.default_rng(404)
    out = {}
    objs = [sg.draw_vehicle(rng, 15.0, 0.0, 12.0, 16, 16) for _ in range(3)]
    objs += [sg.draw_pedestrian(rng, 15.0, 0.0, 2.0, 16, 16) for _ in range(2)]
    out["sixteen_grids_H40"] = sg.Scene(objs, 40, 0.1)
    out["two_vehicles_32_grids_H20"] = sg.Scene([sg.draw_vehicle(rng, 8.0, 0.0, 10.0, 32, 32) for _ in range(2)], 20, 0.1)
    objs = [sg.draw_vehicle(rng, 25.0, 0.0, 15.0, 32, 32) for _ in range(4)]
    objs += [sg.draw_pedestrian(rng, 25.0, 0.0, 2.0, 32, 32) for _ in range(4)]
    out["eight_objects_32_grids_H24"] = sg.Scene(objs, 24, 0.1)
    return out


@pytest.mark.parametrize("name", list(_block_scenes().keys()))
def test_block_units_parity(mhc, ctx, name):
    """Block units (alone and with time splits) against the oracle, and every
    tile variant bit for bit; the host walk of each plan first."""
    s = _block_scenes()[name]
    for v in range(mhc.MHC_N_VARIANTS):
        st, info = mhc.mhc_plan_check(s, v, 5120)
        assert st == mhc.MHC_OK and info["blocked_pairs"] > 0, (name, v, info)
    say(f"block units: {name}")
    o = oracle.evaluate(s, threads=THREADS)
    try:
        ref = None
        for v in range(mhc.MHC_N_VARIANTS):
            mhc.mhc_set_variant(ctx, v)
            g = mhc.mhc_evaluate(ctx, s)
            if ref is None:
                parity.check(s, g, o, f"{name} variant {v}")
                ref = g
            else:
                parity.same_results(ref, g, f"{name} variant {v}")
    finally:
        mhc.mhc_set_variant(ctx, -1)
    assert (o.k64 >= 0).sum() > 100


def _ragged_split_scenes():
    """Scenes with few collision units whose horizons the chosen time split
    does not divide, so the last part of every unit overlaps its neighbour:
    Table I S1 (100 steps, split 8: parts of 13 steps), a prime horizon, and
    all four classes on 30 steps (split 8: parts of 4)."""
    rng = np.random.default_rng(505)
    out = {"table_one_s1": sg.paper_scene(5, n_co=3), "table_one_s1_5_profiles_pip":
           sg.paper_scene(6, n_co=3, n_acc=5, overlap=sg.OVERLAP_PIP)}
    objs = [sg.draw_vehicle(rng, 10.0, 0.0, 12.0, 9, 9) for _ in range(2)]
    objs += [sg.draw_pedestrian(rng, 10.0, 0.0, 2.0, 9, 9)]
    out["prime_horizon_37"] = sg.Scene(objs, 37, 0.1)
    objs = [sg.draw_vehicle(rng, 12.0, 0.0, 12.0, 7, 11) for _ in range(2)]
    objs += [sg.draw_pedestrian(rng, 12.0, 0.0, 2.0, 5, 13) for _ in range(2)]
    out["all_classes_H30"] = sg.Scene(objs, 30, 0.1)
    return out


@pytest.mark.parametrize("name", list(_ragged_split_scenes().keys()))
def test_ragged_time_split_parity(mhc, ctx, name):
    """Time splits whose parts overlap (S does not divide H): against the
    oracle, and every tile variant bit for bit; the host walk of each plan
    first, which also shows that the split is ragged."""
    s = _ragged_split_scenes()[name]
    for v in range(mhc.MHC_N_VARIANTS):
        for waves in (5120, 6144):
            st, info = mhc.mhc_plan_check(s, v, waves)
            assert st == mhc.MHC_OK, (name, v, waves, info)
            if v == 0:      # the default variant, compared with the oracle below
                assert info["time_split"] > 1 and s.horizon % info["time_split"] != 0, (name, waves, info)
    say(f"ragged time split: {name}")
    o = oracle.evaluate(s, threads=THREADS)
    try:
        ref = None
        for v in range(mhc.MHC_N_VARIANTS):
            mhc.mhc_set_variant(ctx, v)
            g = mhc.mhc_evaluate(ctx, s)
            if ref is None:
                parity.check(s, g, o, f"{name} variant {v}")
                ref = g
            else:
                parity.same_results(ref, g, f"{name} variant {v}")
    finally:
        mhc.mhc_set_variant(ctx, -1)
    assert (o.k64 >= 0).sum() > 50


def test_batch_with_different_outputs_per_scene(mhc, ctx):
    """A batch whose scenes ask for different outputs (first hits, q, the
    per-trajectory arrays, the risk over time, each for some scenes only):
    every requested output equals that scene evaluated alone, bit for bit."""
    import ctypes
    scenes = sg.batch_scenes(7, 10)
    for k, s in enumerate(scenes):
        s.timeline = 1 if k % 4 == 1 else 0
    css = [mhc.CScene(s) for s in scenes]
    outs, rs = [], []
    for k, cs in enumerate(css):
        out, r = mhc.host_result(cs, first_hit=k % 2 == 0, q=k % 3 == 0)
        if k % 5 == 2:
            out["traj_crit"], r.traj_crit = None, None
        if k % 3 == 1:
            out["traj_prob"], r.traj_prob = None, None
        outs.append(out)
        rs.append(r)
    arr = (mhc.mhc_scene * len(css))(*[c.c for c in css])
    rarr = (mhc.mhc_result * len(css))(*rs)
    say("batch of 10 scenes with different outputs per scene")
    assert mhc.lib.mhc_evaluate_batch(ctx, len(css), arr, rarr) == mhc.MHC_OK, mhc.mhc_last_error(ctx)
    for k, (s, cs) in enumerate(zip(scenes, css)):
        ref = mhc.mhc_evaluate(ctx, cs, first_hit=True, q=True)
        for name, got in outs[k].items():
            if got is None:
                continue
            assert np.array_equal(got, ref[name].reshape(got.shape)), f"scene {k}: {name}"


def test_size_limits(mhc, ctx):
    """The largest horizon (32767 steps: first hits near the top of the int16
    slot range) and the largest trajectory count of one object (32768)."""
    # two vehicles 66 m apart closing at 0.02 m/s touch after ~30,750 steps
    # of 0.1 s; a slow pedestrian walks towards their meeting point
    s = sg.Scene([veh(0.0, 0.0, 0.0, 0.01, [0.0], [0.0]),
                  veh(66.0, 0.3, math.pi, 0.01, [0.0], [0.0]),
                  ped(33.0, 40.0, -math.pi / 2, 0.02, [0.0, 0.013], [0.0, 0.01])], 32767, 0.1)
    say("horizon 32767")
    g = mhc.mhc_evaluate(ctx, s)
    o = oracle.evaluate(s, threads=THREADS)
    parity.check(s, g, o, "horizon 32767")
    assert int(g["first_hit"][0]) > 25000, g["first_hit"][0]
    # one vehicle with 256 x 128 = 32768 trajectories against a small vehicle
    s = sg.Scene([veh(0.0, 0.0, 0.0, 8.0, sg.accel_grid(256), sg.yaw_grid(128)),
                  veh(9.0, 1.0, 2.8, 3.0, sg.accel_grid(3), sg.yaw_grid(1))], 8, 0.1)
    say("32768 trajectories")
    g = mhc.mhc_evaluate(ctx, s)
    o = oracle.evaluate(s, threads=THREADS)
    parity.check(s, g, o, "32768 trajectories")
    assert (o.k64 >= 0).sum() > 1000 and (o.k64 < 0).sum() > 1000


def test_repeated_shape_reuses_resident_plan(mhc, ctx):
    """Calls on scenes of one shape upload only the value part of the scene
    image while the shape's collision plan is still in the context's
    workspace; a batch, an autotune run or a call of another shape in between
    overwrites it. Every call must equal a fresh context's call on the same
    scene, bit for bit."""
    scenes = [sg.eleven_object_scene(s) for s in range(11, 17)]
    other = sg.paper_scene(7, n_co=3)

    def fresh(scene):
        c = mhc.mhc_create(0)
        try:
            return mhc.mhc_evaluate(c, scene)
        finally:
            mhc.mhc_destroy(c)

    steps = [("evaluate", 0), ("evaluate", 1), ("evaluate", 1), ("batch", None), ("evaluate", 2),
             ("evaluate", 3), ("other", None), ("evaluate", 4), ("autotune", None), ("evaluate", 5),
             ("evaluate", 0)]
    for what, k in steps:
        say(f"resident plan: {what} {k}")
        if what == "batch":
            mhc.mhc_evaluate_batch(ctx, sg.batch_scenes(2, 4), first_hit=False, q=False)
        elif what == "other":
            parity.same_results(mhc.mhc_evaluate(ctx, other), fresh(other), "another shape in between")
        elif what == "autotune":
            mhc.mhc_autotune(ctx, scenes[0], reps=2)
        else:
            parity.same_results(mhc.mhc_evaluate(ctx, scenes[k]), fresh(scenes[k]), f"11-object seed {11 + k}")



def test_repeated_batch_shape_reuses_its_layout(mhc, ctx):
    """Batches of one shape (same scenes' object kinds and grids, new
    positions, speeds and controls) keep the batch layout and upload only the
    image's value part; a single-scene call, a batch of another shape, a
    change of the first-hit request or an autotune run in between rebuild it.
    Every batch must equal a fresh context's batch, bit for bit, scene by
    scene, for several passes (the third repeat of a shape replays a captured
    graph)."""
    import copy
    base = sg.batch_scenes(2, 12)

    def moved(scenes, k):
        out = copy.deepcopy(scenes)
        rng = np.random.default_rng(100 + k)
        for sc in out:
            for o in sc.objects:
                o.x += float(rng.uniform(-3, 3))
                o.y += float(rng.uniform(-3, 3))
                o.speed = max(0.0, o.speed + float(rng.uniform(-1, 1)))
                o.u = o.u * float(rng.uniform(0.9, 1.1))
        return out

    def fresh(scenes, first_hit):
        c = mhc.mhc_create(0)
        try:
            return mhc.mhc_evaluate_batch(c, scenes, first_hit=first_hit)
        finally:
            mhc.mhc_destroy(c)

    steps = [("batch", 0, True), ("batch", 1, True), ("batch", 2, True), ("batch", 3, True),
             ("single", None, True), ("batch", 4, True), ("batch", 5, False), ("batch", 6, False),
             ("other", None, True), ("batch", 7, False), ("autotune", None, True), ("batch", 8, False),
             ("batch", 9, True)]
    for what, k, fh in steps:
        say(f"repeated batch shape: {what} {k} first_hit={fh}")
        if what == "single":
            mhc.mhc_evaluate(ctx, sg.eleven_object_scene(3))
        elif what == "other":
            mhc.mhc_evaluate_batch(ctx, sg.batch_scenes(5, 6), first_hit=False)
        elif what == "autotune":
            mhc.mhc_autotune_batch(ctx, base, reps=1)
        else:
            scenes = moved(base, k)
            got = mhc.mhc_evaluate_batch(ctx, scenes, first_hit=fh)
            want = fresh(scenes, fh)
            for i, (g, w) in enumerate(zip(got, want)):
                parity.same_results(g, w, f"batch pass {k}, scene {i}")
