"""GPU parity over a seeded sweep of random scenes that mix every scene
option (tests/random_scenes.py): object kinds and counts, rectangles and
convex outlines, the three motion models, scores or uniform probabilities,
all or EGO pairs, exact or point-in-polygon overlap, both risk readings, the
risk over time, horizons of 1 to 131 steps (ragged time splits, several
64-step trajectory chunks) and three step lengths. Every scene is checked
against the FP64 oracle by the acceptance rule; some against other tile
variants bit for bit; all of them batched, mixed, against single calls."""
import os

import pytest

import oracle
from tests import parity
from tests.random_scenes import random_scene

pytestmark = pytest.mark.gpu

THREADS = int(os.environ.get("MHC_ORACLE_THREADS", "16"))
N_SCENES = 1000


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


@pytest.fixture(scope="module")
def singles(mhc, ctx):
    """Every scene of the sweep evaluated alone (default tile variant)."""
    say(f"random scenes: {N_SCENES} single calls")
    return [mhc.mhc_evaluate(ctx, random_scene(k)) for k in range(N_SCENES)]


def test_random_scenes_against_the_oracle(mhc, ctx, singles):
    hits = 0
    for k in range(N_SCENES):
        s = random_scene(k)
        o = oracle.evaluate(s, threads=THREADS)
        parity.check(s, singles[k], o, f"random scene {k}")
        hits += int((o.k64 >= 0).sum())
        if k % 5 == 0:
            v = (k // 5) % mhc.MHC_N_VARIANTS
            try:
                mhc.mhc_set_variant(ctx, v)
                parity.same_results(singles[k], mhc.mhc_evaluate(ctx, s), f"random scene {k}, variant {v}")
            finally:
                mhc.mhc_set_variant(ctx, -1)
    say(f"  {hits} colliding trajectory pairs over {N_SCENES} scenes")
    assert hits > 10_000


def test_random_scenes_batched(mhc, ctx, singles):
    say("random scenes: batches of 50, mixed options")
    for b0 in range(0, N_SCENES, 50):
        scenes = [random_scene(k) for k in range(b0, b0 + 50)]
        for k, g in enumerate(mhc.mhc_evaluate_batch(ctx, scenes)):
            parity.same_results(singles[b0 + k], g, f"random scene {b0 + k} in a batch")
