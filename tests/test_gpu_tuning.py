"""GPU tests of the tile-variant autotuner: tuning a single scene and a
batch, the save -> load round trip of the tune file (including files from
before the scene-count field), rejection of malformed files without any
change, and results that do not depend on the variant chosen."""
import os

import numpy as np
import pytest

from paper_2005_06773_amd import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def mhc():
    from paper_2005_06773_amd import mhc as m
    return m


def test_tune_round_trip_and_batch_tuning(mhc, tmp_path):
    a = mhc.mhc_create(0)
    b = mhc.mhc_create(0)
    try:
        scene = sg.eleven_object_scene(1)
        batch = sg.batch_scenes(2, 16)
        say("autotune: 11-object scene and a 16-scene batch")
        best1, us1 = mhc.mhc_autotune(a, scene, reps=3)
        bestb, usb = mhc.mhc_autotune_batch(a, batch, reps=2)
        assert 0 <= best1 < mhc.MHC_N_VARIANTS and 0 <= bestb < mhc.MHC_N_VARIANTS
        assert all(u > 0 for u in us1 + usb)
        assert usb[bestb] == min(usb) and us1[best1] == min(us1)
        say(f"  single scene variant {best1} {['%.1f' % u for u in us1]} us; batch variant {bestb} "
            f"{['%.1f' % u for u in usb]} us")
        path_a = str(tmp_path / "tune_a.json")
        mhc.mhc_tune_save(a, path_a)
        text = open(path_a).read()
        assert text.startswith('{"gfx950": {') and text.count(":") == 3, text   # two classes
        # the batch is a class of its own (scene-count bucket 4 for 16 scenes)
        assert ',4": ' in text and ',0": ' in text, text
        mhc.mhc_tune_load(b, path_a)
        path_b = str(tmp_path / "tune_b.json")
        mhc.mhc_tune_save(b, path_b)
        assert open(path_b).read() == text
        # batched results are the same with the tuned and the default variant
        tuned = mhc.mhc_evaluate_batch(b, batch)
        plain = mhc.mhc_create(0)
        try:
            for k, (x, y) in enumerate(zip(tuned, mhc.mhc_evaluate_batch(plain, batch))):
                parity.same_results(x, y, f"batch scene {k}, tuned vs default variant")
        finally:
            mhc.mhc_destroy(plain)
        # files written before the scene-count (and family) fields existed
        old = tmp_path / "old.json"
        old.write_text('{"gfx950": {"3,2": 1, "5,3,1": 2}}\n')
        mhc.mhc_tune_load(b, str(old))
        mhc.mhc_tune_save(b, path_b)
        new = open(path_b).read()
        assert '"3,2,0,0": 1' in new and '"5,3,1,0": 2' in new, new
        # malformed files are refused and change nothing
        bad_files = {"no_arch.json": '{"gfx942": {"3,2,0,0": 1}}',
                     "bad_variant.json": '{"gfx950": {"3,2,0,0": 1, "4,4,0,0": 9}}',
                     "garbage.json": '{"gfx950": {"x,y": one}}',
                     "unclosed.json": '{"gfx950": '}
        for name, body in bad_files.items():
            p = tmp_path / name
            p.write_text(body)
            with pytest.raises(mhc.MhcError) as ei:
                mhc.mhc_tune_load(b, str(p))
            assert ei.value.status == mhc.MHC_E_INVAL, name
            assert mhc.mhc_last_error(b)
            mhc.mhc_tune_save(b, path_b)
            assert open(path_b).read() == new, f"{name} changed the tuned choices"
        with pytest.raises(mhc.MhcError):
            mhc.mhc_tune_load(b, str(tmp_path / "does_not_exist.json"))
        with pytest.raises(mhc.MhcError):
            mhc.mhc_autotune_batch(b, [], reps=1)
    finally:
        mhc.mhc_destroy(a)
        mhc.mhc_destroy(b)


def test_server_keeps_its_tuning_snapshot(mhc):
    """A server copies the context's variant choices when it starts; retuning
    or forcing a variant on the context meanwhile changes neither its results
    nor the context's own."""
    ctx = mhc.mhc_create(0)
    try:
        scenes = sg.batch_scenes(5, 12)
        ref = [mhc.mhc_evaluate(ctx, s) for s in scenes]
        srv = mhc.Server(ctx, budget=1 << 30)
        tickets = []
        for k, s in enumerate(scenes):
            tickets.append(srv.submit(0, s, first_hit=True, q=True))
            mhc.mhc_set_variant(ctx, k % mhc.MHC_N_VARIANTS)          # the context's own thread
            parity.same_results(ref[k], mhc.mhc_evaluate(ctx, s), f"context call {k} while serving")
        outs = [srv.wait(t)[0] for t in tickets]
        srv.stop()
        for k, o in enumerate(outs):
            parity.same_results(ref[k], o, f"served frame {k}")
    finally:
        mhc.mhc_set_variant(ctx, -1)
        mhc.mhc_destroy(ctx)


def test_autotune_one_variant_at_a_time_under_a_budget(mhc):
    """With a context budget that holds one variant's image but not all four
    together, the tuner times the variants one at a time in the context
    workspace; it still returns a time for every variant and records the
    fastest, and results stay those of the default variant."""
    scene = sg.eleven_object_scene(1)
    cs = mhc.CScene(scene)
    # 8.2 MB with the 5.6 MB of first hits the evaluation asks for; the tuner's
    # images (no first hits) are about 2.6 MB each, 10.5 MB for all four
    need = mhc.mhc_query_sizes(cs)["device_bytes"]
    small = mhc.mhc_create(0, int(need * 1.05))
    free = mhc.mhc_create(0)
    try:
        say(f"autotune under a {need * 1.05 / 1e6:.1f} MB budget")
        best, us = mhc.mhc_autotune(small, scene, reps=3)
        assert 0 <= best < mhc.MHC_N_VARIANTS and len(us) == mhc.MHC_N_VARIANTS
        assert all(u > 0 for u in us) and us[best] == min(us)
        say(f"  variant {best} {['%.1f' % u for u in us]} us")
        parity.same_results(mhc.mhc_evaluate(free, scene), mhc.mhc_evaluate(small, scene),
                            "tuned under a budget vs default")
    finally:
        mhc.mhc_destroy(small)
        mhc.mhc_destroy(free)
