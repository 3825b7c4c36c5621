"""Pins of the oracle's trajectories (Sec. IV-B.1, IV-B.3), pair counts
(Sec. IV-B.4, IV-C.2, Table I), first hits and risk (Sec. IV-D, IV-D.2)."""
import math

import numpy as np
import pytest

import oracle
from paper_2005_06773_amd import scenegen as sg


def veh(x, y, psi, v, u, w, L=4.5, W=1.8, score=None):
    return sg.SceneObject(sg.VEHICLE, x, y, psi, v, L, W, 0.0, np.asarray(u, float), np.asarray(w, float), score)


def ped(x, y, psi, v, u, w, r=0.3, score=None):
    return sg.SceneObject(sg.PEDESTRIAN, x, y, psi, v, 0.0, 0.0, r, np.asarray(u, float), np.asarray(w, float), score)


def _golden():
    import os
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, val = line.split()[:2]
            vals[name] = int(val)
    return vals


# --------------------------------------------------------------------------
# Counts printed in the paper
# --------------------------------------------------------------------------

def test_paper_trajectory_and_combination_counts():
    g = _golden()
    s2 = sg.paper_shaped_sizes(10)
    assert s2[0] == g["ego_trajectories"] and s2[1] == g["co_trajectories"]
    assert oracle.count_trajectories(s2) == g["r_tra_o10"]
    assert oracle.count_combinations(s2, ego_only=True) == g["r_col_o10"]
    H = g["horizon_steps"]
    assert 2 * H * oracle.count_combinations(s2, True) == g["overlap_calls_s2"]
    per_co = oracle.count_combinations(sg.paper_shaped_sizes(1), True) * H
    assert round(per_co / 1e4) * 1e4 == g["pose_combinations_per_co"]
    s1 = sg.paper_shaped_sizes(3)
    assert round(oracle.count_combinations(s1, True) * H / 1e4) * 1e4 == g["pose_combinations_s1_6"]
    assert round(oracle.count_combinations(s2, True) * H / 1e4) * 1e4 == g["pose_combinations_s2_6"]
    # the 5-profile figures are printed 0.0075 M / 0.015 M below the formula
    s1_5 = sg.paper_shaped_sizes(3, n_acc=5)
    s2_5 = sg.paper_shaped_sizes(10, n_acc=5)
    assert abs(oracle.count_combinations(s1_5, True) * H - g["pose_combinations_s1_5"]) <= 2e4
    assert abs(oracle.count_combinations(s2_5, True) * H - g["pose_combinations_s2_5"]) <= 2e4


def test_pair_enumeration():
    assert oracle.pairs(4, False) == [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    assert oracle.pairs(4, True) == [(0, 1), (0, 2), (0, 3)]
    assert len(oracle.pairs(11, False)) == 55
    assert len(oracle.pairs(40, False)) == 780
    # the 11-object scene: 83,531,250 pose-pair checks
    s = sg.eleven_object_scene(1)
    assert oracle.count_combinations(s.traj_counts(), False) * s.horizon == 83_531_250
    st = sg.stress_scene()
    assert oracle.count_combinations(st.traj_counts(), False) * st.horizon == 40_894_464_000


# --------------------------------------------------------------------------
# Probabilities
# --------------------------------------------------------------------------

def test_probabilities_l1_normalised():
    s = sg.eleven_object_scene(3)
    for o in s.objects:
        p = oracle.probabilities(o)
        assert abs(p.sum() - 1.0) < 1e-14 and (p >= 0).all()
        assert np.allclose(p * o.score.sum(), o.score, rtol=1e-14)
    o = veh(0, 0, 0, 1, [0, 1, 2], [0, 1])
    assert np.all(oracle.probabilities(o) == 1.0 / 6)


def test_probabilities_reject_invalid():
    for bad in ([0.0, 0.0], [1.0, -0.5], [1.0, np.nan], [np.inf, 1.0]):
        o = veh(0, 0, 0, 1, [0, 1], [0], score=np.array(bad))
        with pytest.raises(ValueError):
            oracle.probabilities(o)


# --------------------------------------------------------------------------
# Trajectories
# --------------------------------------------------------------------------

def test_straight_line_at_constant_speed():
    o = veh(3.0, -2.0, 0.7, 12.0, [0.0], [0.0])
    x, y, psi = oracle.trajectories(o, 40, 0.1)
    n = np.arange(1, 41)
    assert np.allclose(x[:, 0], 3.0 + n * 0.1 * 12.0 * math.cos(0.7), atol=1e-11)
    assert np.allclose(y[:, 0], -2.0 + n * 0.1 * 12.0 * math.sin(0.7), atol=1e-11)
    assert np.allclose(psi[:, 0], 0.7, atol=0)


def test_constant_acceleration_is_exact():
    """The step update integrates a constant acceleration exactly: the
    position after n steps is v0 t + a t^2 / 2 along the heading."""
    o = veh(0.0, 0.0, 1.1, 5.0, [2.5], [0.0])
    x, y, _ = oracle.trajectories(o, 30, 0.1)
    t = np.arange(1, 31) * 0.1
    s = 5.0 * t + 2.5 * t * t / 2
    assert np.allclose(x[:, 0], s * math.cos(1.1), atol=1e-11)
    assert np.allclose(y[:, 0], s * math.sin(1.1), atol=1e-11)


def test_braking_stops_and_stays():
    """a = -8 m/s^2 from 10 m/s with 0.1 s steps: speeds 10, 9.2, ..., 0.4
    after 12 steps, then the vehicle stops within step 13, which advances it
    by 0.4 * 0.1 / 2 m: 6.24 + 0.02 = 6.26 m in total, constant afterwards."""
    o = veh(0.0, 0.0, 0.0, 10.0, [-8.0], [0.0])
    x, y, _ = oracle.trajectories(o, 30, 0.1)
    assert x[11, 0] == pytest.approx(6.24, abs=1e-12)
    assert x[12, 0] == pytest.approx(6.26, abs=1e-12)
    assert np.all(x[12:, 0] == x[12, 0])
    assert np.all(y[:, 0] == 0.0)


def test_constant_turn_follows_circle_to_second_order():
    """At constant speed v and yaw rate w the exact path is a circular arc of
    radius v/w; the second-order step update stays within O(tau^2) of it and
    the error falls by ~4x when tau halves."""
    v, w, T_end = 10.0, 0.5, 3.0
    errs = []
    for tau in (0.02, 0.01):
        H = int(round(T_end / tau))
        o = veh(0.0, 0.0, 0.0, v, [0.0], [w])
        x, y, psi = oracle.trajectories(o, H, tau)
        t = np.arange(1, H + 1) * tau
        xe, ye = (v / w) * np.sin(w * t), (v / w) * (1 - np.cos(w * t))
        errs.append(np.max(np.hypot(x[:, 0] - xe, y[:, 0] - ye)))
        assert np.allclose(psi[:, 0], w * t, atol=1e-12)
    assert errs[0] < 2e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_yaw_rate_sign_mirrors_path():
    o = veh(0.0, 0.0, 0.0, 8.0, [1.0], [-0.3, 0.3])
    x, y, _ = oracle.trajectories(o, 30, 0.1)
    assert np.allclose(x[:, 0], x[:, 1], atol=1e-12)
    assert np.allclose(y[:, 0], -y[:, 1], atol=1e-12)


def test_pedestrian_linear_in_steps():
    o = ped(1.0, 2.0, 0.3, 1.2, [0.0, 1.0, 2.5], [0.0, math.pi / 2])
    x, y, psi = oracle.trajectories(o, 25, 0.1)
    n = np.arange(1, 26) * 0.1
    for k, s in enumerate([0.0, 1.0, 2.5]):
        for l, h in enumerate([0.0, math.pi / 2]):
            i = k * 2 + l
            assert np.allclose(x[:, i], 1.0 + n * s * math.cos(0.3 + h), atol=1e-12)
            assert np.allclose(y[:, i], 2.0 + n * s * math.sin(0.3 + h), atol=1e-12)


def test_trajectory_index_order():
    """Trajectory i = k*n_w + l uses u[k] and w[l]."""
    o = veh(0, 0, 0, 10.0, [-4.0, 0.0, 2.0], [-0.2, 0.2])
    x, y, psi = oracle.trajectories(o, 10, 0.1)
    for k, a in enumerate([-4.0, 0.0, 2.0]):
        for l, w in enumerate([-0.2, 0.2]):
            single = veh(0, 0, 0, 10.0, [a], [w])
            xs, ys, ps = oracle.trajectories(single, 10, 0.1)
            assert np.array_equal(x[:, k * 2 + l], xs[:, 0])
            assert np.array_equal(psi[:, k * 2 + l], ps[:, 0])


# --------------------------------------------------------------------------
# First hits
# --------------------------------------------------------------------------

def test_head_on_first_hit_closed_form():
    """Two vehicles on one line, heading at each other at v1 and v2: the
    first colliding step is n* = ceil((D - (L1+L2)/2) / ((v1+v2) tau)),
    stored at slot n* - 1."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        D = rng.uniform(20, 80)
        v1, v2 = rng.uniform(1, 20, 2)
        L1, L2 = rng.uniform(3, 6, 2)
        tau = 0.1
        A = veh(0.0, 0.0, 0.0, v1, [0.0], [0.0], L=L1)
        B = veh(D, 0.0, math.pi, v2, [0.0], [0.0], L=L2)
        gap_steps = (D - (L1 + L2) / 2) / ((v1 + v2) * tau)
        if abs(gap_steps - round(gap_steps)) < 1e-6:
            continue
        H = int(math.ceil(gap_steps)) + 5
        r = oracle.evaluate(sg.Scene([A, B], H, tau), masks=False)
        assert r.k64[0] == math.ceil(gap_steps) - 1


def test_stationary_pair_constant_overlap():
    for dx, expect in ((3.0, 0), (6.0, -1)):
        A = veh(0.0, 0.0, 0.0, 0.0, [0.0, -3.0], [0.0, 0.2])
        B = veh(dx, 0.0, 0.0, 0.0, [0.0], [0.0])
        r = oracle.evaluate(sg.Scene([A, B], 20, 0.1))
        assert r.k64[0] == expect          # (a=0, w=0): never moves
        assert r.k64[1] == expect          # (a=0, w=0.2): rotates in place
        assert r.k64[2] == expect          # braking from rest: stays
    # at 4.6 m the rectangle turning in place sweeps its corner into B
    A = veh(0.0, 0.0, 0.0, 0.0, [0.0], [0.2])
    B = veh(4.6, 0.0, 0.0, 0.0, [0.0], [0.0])
    assert oracle.evaluate(sg.Scene([A, B], 20, 0.1)).k64[0] > 0


def test_swap_symmetry_transposes_first_hits():
    s = sg.eleven_object_scene(7)
    s.objects = s.objects[:3] + s.objects[6:8]
    r = oracle.evaluate(s, masks=False)
    rev = sg.Scene(list(reversed(s.objects)), s.horizon, s.dt)
    rr = oracle.evaluate(rev, masks=False)
    n = len(s.objects)
    T = s.traj_counts()
    for p, (a, b) in enumerate(zip(r.pair_a, r.pair_b)):
        blk = r.k64[r.pair_off[p]:r.pair_off[p + 1]].reshape(T[a], T[b])
        ra, rb = n - 1 - b, n - 1 - a
        q = [k for k, (x, y) in enumerate(zip(rr.pair_a, rr.pair_b)) if (x, y) == (ra, rb)][0]
        blk2 = rr.k64[rr.pair_off[q]:rr.pair_off[q + 1]].reshape(T[b], T[a])
        assert np.array_equal(blk, blk2.T)
    assert np.allclose(r.obj_crit, rr.obj_crit[::-1], atol=1e-15)


# --------------------------------------------------------------------------
# Risk
# --------------------------------------------------------------------------

def _colliding_scene(seed, n=5):
    rng = np.random.default_rng(seed)
    objs = []
    for k in range(n):
        if k < 3:
            objs.append(veh(rng.uniform(-8, 8), rng.uniform(-8, 8), rng.uniform(0, 6.28), rng.uniform(2, 10),
                            sg.accel_grid(5), sg.yaw_grid(4), score=rng.uniform(0.1, 1.0, 20)))
        else:
            objs.append(ped(rng.uniform(-6, 6), rng.uniform(-6, 6), rng.uniform(0, 6.28), 1.0,
                            sg.ped_speed_grid(4), sg.ped_heading_grid(5), score=rng.uniform(0.1, 1.0, 20)))
    return sg.Scene(objs, 25, 0.1)


def test_single_collision_object_reduces_to_double_sum():
    """With one collision object, C_EGO is the paper's p_cra =
    sum_i sum_j I(i,j) p_EGO,i p_CO,j (Sec. IV-D)."""
    n_with_hits = 0
    for seed in range(12):
        s = _colliding_scene(seed, n=5)
        s.objects = s.objects[:2]
        r = oracle.evaluate(s)
        I = (r.k64 >= 0).reshape(s.objects[0].n_traj, s.objects[1].n_traj)
        pe, pc = oracle.probabilities(s.objects[0]), oracle.probabilities(s.objects[1])
        p_cra = float(np.sum(I * pe[:, None] * pc[None, :]))
        assert r.obj_crit[0] == pytest.approx(p_cra, abs=1e-15)
        n_with_hits += bool(I.any())
    assert n_with_hits >= 3


def test_chronological_scaling_telescopes():
    """Sec. IV-D.2: the earliest combination counts in full, each later one
    is multiplied by the chance that none before it collided. Summing
    these in the chronological order of each object's earliest hit gives the
    oracle's 1 - prod(1 - q), in any order."""
    s = _colliding_scene(21, n=6)
    r = oracle.evaluate(s)
    n = s.n_objects
    T = s.traj_counts()
    toff = np.concatenate([[0], np.cumsum(T)])
    first = {}
    for p, (a, b) in enumerate(zip(r.pair_a, r.pair_b)):
        blk = r.k64[r.pair_off[p]:r.pair_off[p + 1]].reshape(T[a], T[b])
        big = np.where(blk >= 0, blk, 10 ** 6)
        first[(a, b)] = big.min(axis=1)
        first[(b, a)] = big.min(axis=0)
    rng = np.random.default_rng(0)
    checked = 0
    for a in range(n):
        for i in range(T[a]):
            others = [b for b in range(n) if b != a]
            order = sorted(others, key=lambda b: (first[(a, b)][i], b))
            for perm in (order, list(rng.permutation(others))):
                total, keep = 0.0, 1.0
                for b in perm:
                    qb = r.q[toff[a] + i, b]
                    total += keep * qb
                    keep *= (1.0 - qb)
                assert total == pytest.approx(r.traj_crit[toff[a] + i], abs=1e-14)
            checked += r.traj_crit[toff[a] + i] > 0
    assert checked > 10


def test_risk_bounds_and_monotonicity():
    s = _colliding_scene(5, n=6)
    r = oracle.evaluate(s)
    assert np.all((r.traj_crit >= 0) & (r.traj_crit <= 1))
    assert np.all((r.obj_crit >= 0) & (r.obj_crit <= 1))
    assert np.all((r.q >= 0) & (r.q <= 1))
    # adding an object never lowers the criticality of the others
    s_less = sg.Scene(s.objects[:-1], s.horizon, s.dt)
    r_less = oracle.evaluate(s_less)
    assert np.all(r.obj_crit[:-1] >= r_less.obj_crit - 1e-15)
    assert r.obj_crit.max() > 0


def test_ego_mode_matches_all_pairs_for_ego():
    s = _colliding_scene(8, n=5)
    r_all = oracle.evaluate(s)
    s_ego = sg.Scene(s.objects, s.horizon, s.dt, pairs=sg.PAIRS_EGO)
    r_ego = oracle.evaluate(s_ego)
    assert len(r_ego.pair_a) == 4
    assert r_ego.obj_crit[0] == pytest.approx(r_all.obj_crit[0], abs=0)
    T0 = s.objects[0].n_traj
    assert np.array_equal(r_ego.traj_crit[:T0], r_all.traj_crit[:T0])


def test_relabelling_permutes_criticality():
    s = _colliding_scene(13, n=5)
    r = oracle.evaluate(s)
    perm = [0, 3, 1, 4, 2]
    sp = sg.Scene([s.objects[k] for k in perm], s.horizon, s.dt)
    rp = oracle.evaluate(sp)
    assert np.allclose(rp.obj_crit, r.obj_crit[perm], atol=1e-15)


def test_acceptance_rule():
    """Bit equality with k64 is always accepted; shifting a first hit that is
    clear of the band is rejected."""
    s = _colliding_scene(2, n=4)
    r = oracle.evaluate(s)
    assert oracle.accepted_first_hits(r.k64, r).all()
    clear = (r.k64 >= 0) & (r.kstrict == r.k64)
    assert clear.any()
    bad = r.k64.copy()
    bad[clear] += 1
    assert not oracle.accepted_first_hits(bad, r)[clear].any()
    bad = r.k64.copy()
    bad[clear] = -1
    assert not oracle.accepted_first_hits(bad, r)[clear].any()
