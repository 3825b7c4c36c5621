"""GPU parity of general convex vehicle outlines (Sec. IV-C.1) through the C
ABI against the FP64 oracle: octagonal cars in the 11-object scene, random
outlines of 3 to 8 vertices with pedestrians, both overlap modes, outlines
that equal the rectangle (against the rectangle path, bit for bit), every
tile variant, batches and the risk over time."""
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


def random_outline_scene(seed, n_veh=5, n_ped=3, horizon=30, overlap=sg.OVERLAP_EXACT):
    """Vehicles with random convex outlines (3..8 vertices, some offset from
    the tracked point) and pedestrians, close together so that many
    combinations collide."""
    rng = np.random.default_rng(seed)
    objs = []
    for k in range(n_veh):
        o = sg.draw_vehicle(rng, 12.0, 0.0, 10.0, int(rng.integers(3, 9)), int(rng.integers(3, 9)))
        out = sg.random_convex_outline(rng, int(rng.integers(3, 9)), rng.uniform(0.6, 1.2), rng.uniform(1.5, 2.5))
        if k % 3 == 2:
            out = out - [out[:, 0].max() + 0.5, 0.0]   # all behind the tracked point, like a trailer
        o.outline = out
        objs.append(o)
    if overlap == sg.OVERLAP_EXACT:
        for _ in range(n_ped):
            objs.append(sg.draw_pedestrian(rng, 12.0, 0.0, 2.0, int(rng.integers(2, 6)), int(rng.integers(3, 8))))
    return sg.Scene(objs, horizon, 0.1, overlap=overlap)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_octagon_cars_parity(mhc, ctx, seed):
    s = sg.polygon_scene(seed)
    say(f"11-object scene with octagonal cars, seed {seed}")
    g = mhc.mhc_evaluate(ctx, s)
    o = oracle.evaluate(s, threads=THREADS)
    parity.check(s, g, o, f"octagons seed {seed}")
    assert (o.k64 >= 0).sum() > 1000


@pytest.mark.parametrize("seed", range(6))
def test_random_outlines_parity(mhc, ctx, seed):
    s = random_outline_scene(100 + seed)
    say(f"random outlines with pedestrians, seed {100 + seed}")
    parity.check(s, mhc.mhc_evaluate(ctx, s), oracle.evaluate(s, threads=THREADS), f"random outlines {seed}")


@pytest.mark.parametrize("seed", range(3))
def test_random_outlines_point_in_polygon_parity(mhc, ctx, seed):
    s = random_outline_scene(200 + seed, n_veh=7, overlap=sg.OVERLAP_PIP)
    say(f"random outlines, point-in-polygon, seed {200 + seed}")
    o = oracle.evaluate(s, threads=THREADS)
    parity.check(s, mhc.mhc_evaluate(ctx, s), o, f"random outlines pip {seed}")
    assert (o.k64 >= 0).any()


def test_table_one_octagons_both_modes(mhc, ctx):
    for overlap in (sg.OVERLAP_EXACT, sg.OVERLAP_PIP):
        s = sg.paper_scene(5, n_co=3, overlap=overlap)
        for ob in s.objects:
            ob.outline = sg.car_outline(ob.length, ob.width)
        say(f"Table I S1 with octagonal cars, overlap {overlap}")
        parity.check(s, mhc.mhc_evaluate(ctx, s), oracle.evaluate(s, threads=THREADS), f"Table I octagons {overlap}")


def test_rectangle_outlines_equal_the_rectangle_path(mhc, ctx):
    """A vehicle whose outline is its own rectangle goes through the polygon
    test; its first hits must equal those of the rectangle test (both exact
    modes agree with the oracle, and here with each other entry by entry)."""
    for overlap in (sg.OVERLAP_EXACT, sg.OVERLAP_PIP):
        s = sg.eleven_object_scene(5)
        if overlap == sg.OVERLAP_PIP:
            s.objects = s.objects[:6]
        s.overlap = overlap
        ref = mhc.mhc_evaluate(ctx, s)
        for ob in s.objects:
            if ob.kind == sg.VEHICLE:
                l, w = ob.length / 2, ob.width / 2
                ob.outline = np.array([[l, -w], [l, w], [-l, w], [-l, -w]])
        got = mhc.mhc_evaluate(ctx, s)
        o = oracle.evaluate(s, threads=THREADS)
        parity.check(s, got, o, f"rectangle outlines {overlap}")
        same = np.mean(ref["first_hit"] == got["first_hit"])
        say(f"  overlap {overlap}: first hits equal to the rectangle path: {same:.7f}")
        amb = (o.kstrict != o.k64) | (oracle.first_loose_slot(o.loose) != o.k64)
        assert np.array_equal(ref["first_hit"][~amb], got["first_hit"][~amb])


def test_one_outline_among_rectangles(mhc, ctx):
    """Only the EGO has an outline: its pairs are polygon pairs (the others'
    rectangles as polygons), the rest stay rectangle and circle pairs."""
    s = sg.eleven_object_scene(6)
    s.objects[0].outline = sg.car_outline(s.objects[0].length, s.objects[0].width, 0.5)
    parity.check(s, mhc.mhc_evaluate(ctx, s), oracle.evaluate(s, threads=THREADS), "one outline")


def test_every_tile_variant_is_identical_on_polygons(mhc, ctx):
    scenes = [sg.polygon_scene(3), random_outline_scene(300),
              random_outline_scene(301, n_veh=6, overlap=sg.OVERLAP_PIP)]
    for k, s in enumerate(scenes):
        ref = None
        for v in range(mhc.MHC_N_VARIANTS):
            mhc.mhc_set_variant(ctx, v)
            got = mhc.mhc_evaluate(ctx, s)
            if ref is None:
                ref = got
                parity.check(s, got, oracle.evaluate(s, threads=THREADS), f"scene {k} variant {v}")
            parity.same_results(ref, got, f"scene {k} variant {v}")
    mhc.mhc_set_variant(ctx, -1)


def test_batch_and_timeline_with_outlines(mhc, ctx):
    scenes = sg.batch_scenes(21, 12)
    rng = np.random.default_rng(21)
    for k, s in enumerate(scenes):
        if k % 2:
            for ob in s.objects:
                if ob.kind == sg.VEHICLE and rng.uniform() < 0.7:
                    ob.outline = sg.car_outline(ob.length, ob.width, rng.uniform(0.1, 0.6))
        s.timeline = 1 if k % 3 == 0 else 0
    outs = mhc.mhc_evaluate_batch(ctx, scenes)
    for k, s in enumerate(scenes):
        parity.same_results(mhc.mhc_evaluate(ctx, s), outs[k], f"batch scene {k}")
    s = sg.polygon_scene(4)
    s.timeline = 1
    say("octagon scene with the risk over time")
    parity.check(s, mhc.mhc_evaluate(ctx, s), oracle.evaluate(s, threads=THREADS), "octagons timeline")
