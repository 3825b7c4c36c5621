"""GPU tests of the serving form (continuous batching).

Each frame's results must be identical (first hits and criticality, bit for
bit) to an evaluation of the same scene alone, whatever tick carried it and
whatever else was in that tick; admission must respect the HBM budget.
"""
import threading
import time

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


def test_frames_identical_alone_and_in_the_mix(mhc, ctx):
    scenes = sg.batch_scenes(7, 48)
    alone = [mhc.mhc_evaluate(ctx, s) for s in scenes]
    say("server: 4 producer threads x 12 frames, Poisson-like gaps")
    srv = mhc.Server(ctx, budget=1 << 30, inflight=2)
    results = {}
    errors = []

    def producer(k):
        rng = np.random.default_rng(100 + k)
        try:
            tickets = []
            for j in range(k, len(scenes), 4):
                tickets.append((j, srv.submit(k, scenes[j], first_hit=True, q=True)))
                time.sleep(float(rng.exponential(0.002)))
            for j, t in tickets:
                out, timing = srv.wait(t)
                assert timing["submit_ns"] <= timing["admit_ns"] <= timing["launch_ns"] <= timing["done_ns"]
                results[j] = out
        except Exception as e:  # noqa: BLE001
            errors.append(e)

    threads = [threading.Thread(target=producer, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    st = srv.stats()
    srv.stop()
    assert not errors, errors
    assert len(results) == len(scenes)
    for j in range(len(scenes)):
        parity.same_results(alone[j], results[j], f"frame {j}")
    say(f"  stats: ticks {st['ticks']}, p50 {st['p50_ms']:.3f} ms, p99 {st['p99_ms']:.3f} ms")
    assert st["completed"] == len(scenes) and st["ticks"] >= 2 and st["p99_ms"] >= st["p50_ms"] > 0


def test_served_frames_match_oracle(mhc, ctx):
    scenes = [s for s in sg.batch_scenes(11, 24)][:6]
    srv = mhc.Server(ctx, budget=256 << 20)
    tickets = [srv.submit(0, s, first_hit=True, q=True) for s in scenes]
    outs = [srv.wait(t)[0] for t in tickets]
    srv.stop()
    for k, (s, g) in enumerate(zip(scenes, outs)):
        if sum(o.n_traj for o in s.objects) ** 2 * s.horizon > 2e9:
            continue
        parity.check(s, g, oracle.evaluate(s, threads=16), f"served frame {k}")


def test_budget_admission(mhc, ctx):
    big = sg.eleven_object_scene(1)
    small = sg.two_vehicle_scene(3)
    # a budget below one 11-object frame with its 5.6 MB first-hit output:
    # that frame is refused, small ones pass
    srv = mhc.Server(ctx, budget=4 << 20, inflight=1)
    with pytest.raises(mhc.MhcError) as ei:
        srv.submit(0, big, first_hit=True)
    assert ei.value.status == mhc.MHC_E_NOMEM
    t = srv.submit(0, small, first_hit=True)
    out, _ = srv.wait(t)
    parity.same_results(mhc.mhc_evaluate(ctx, small), out, "small frame under a tiny budget")
    st = srv.stats()
    srv.stop()
    assert st["rejected"] == 1 and st["completed"] == 1
    # a budget that holds one such frame per tick (8.5 MB reserved for it, in
    # slots of 9 MiB less the slot table): frames wait for later ticks
    srv = mhc.Server(ctx, budget=18 << 20, inflight=2)
    ts = [srv.submit(0, big, first_hit=True) for _ in range(6)]
    outs = [srv.wait(t)[0] for t in ts]
    st = srv.stats()
    srv.stop()
    ref = mhc.mhc_evaluate(ctx, big, first_hit=False, q=False)
    for o in outs:
        assert np.array_equal(o["object_crit"], ref["object_crit"])
    assert st["ticks"] >= 3 and st["deferred"] >= 1


def test_wait_timeout_keeps_ticket(mhc, ctx):
    srv = mhc.Server(ctx, budget=1 << 30)
    t = srv.submit(0, sg.stress_scene(4))
    with pytest.raises(mhc.MhcError) as ei:
        srv.wait(t, timeout_us=0)
    assert ei.value.status == mhc.MHC_E_TIMEOUT
    out, timing = srv.wait(t)
    assert np.all(np.isfinite(out["object_crit"]))
    srv.stop()


def test_invalid_frame_rejected(mhc, ctx):
    srv = mhc.Server(ctx, budget=64 << 20)
    s = sg.two_vehicle_scene(0)
    s.dt = -1.0
    with pytest.raises(mhc.MhcError) as ei:
        srv.submit(0, s)
    assert ei.value.status == mhc.MHC_E_INVAL
    srv.stop()


def test_poisson_schedule_frames_alone_and_in_the_mix(mhc, ctx):
    """Frames of the serving workload (32 streams, each a Poisson process at
    10 Hz, frames drawn as in the batch workload), submitted at their
    scheduled arrival times over one second: each frame's results equal the
    same scene evaluated alone, bit for bit, whatever else its tick carried."""
    events = sg.serving_schedule(3, streams=32, rate_hz=10.0, duration_s=1.0, warmup_s=0.0)
    say(f"serving schedule: {len(events)} frames over 1 s from 32 streams")
    srv = mhc.Server(ctx, budget=2 << 30, inflight=2)
    tickets = []
    t0 = time.perf_counter()
    for t_arr, stream, scene in events:
        delay = t_arr - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(stream, scene, first_hit=True, q=True))
    outs = [srv.wait(t)[0] for t in tickets]
    st = srv.stats()
    srv.stop()
    say(f"  ticks {st['ticks']}, frames per tick {len(events) / max(1, st['ticks']):.2f}, "
        f"p50 {st['p50_ms']:.3f} ms, p99 {st['p99_ms']:.3f} ms")
    for k, ((_, stream, scene), out) in enumerate(zip(events, outs)):
        parity.same_results(mhc.mhc_evaluate(ctx, scene), out, f"frame {k} of stream {stream}")
    assert st["completed"] == len(events)


def test_large_frames_run_in_parts(mhc, ctx):
    """With a small per-tick check cap, 11-object frames (83.5 M checks) ride
    alone and their collision plan runs as nine launches, while small frames
    share the other slot: every frame equals the scene evaluated alone."""
    big = [sg.eleven_object_scene(s) for s in (1, 2)]
    small = [sg.two_vehicle_scene(s) for s in range(4)]
    four = sg.eleven_object_scene(3)          # 2 vehicles, 2 pedestrians: 9.1 M checks
    four.objects = four.objects[:2] + four.objects[6:8]
    small.append(four)
    say(f"large frames in parts: 2 x 83.5 M checks with cap 1e7, {len(small)} small frames")
    srv = mhc.Server(ctx, budget=1 << 30, inflight=2, checks_per_tick=10_000_000)
    tb = [srv.submit(0, s, first_hit=True, q=True) for s in big]
    ts = [srv.submit(1, s, first_hit=True, q=True) for s in small]
    outs_b = [srv.wait(t)[0] for t in tb]
    outs_s = [srv.wait(t)[0] for t in ts]
    srv.stop()
    for k, (s, o) in enumerate(zip(big, outs_b)):
        parity.same_results(mhc.mhc_evaluate(ctx, s), o, f"large frame {k}")
    for k, (s, o) in enumerate(zip(small, outs_s)):
        parity.same_results(mhc.mhc_evaluate(ctx, s), o, f"small frame {k}")
