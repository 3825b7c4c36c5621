"""Pins of the oracle's risk readings and of its risk over time (Sec. IV-D,
Sec. IV-D.2, the anticipation time of Sec. VI-A).

The oracle takes the chronological scaling literally, one colliding
combination at a time. These tests pin it to things other than itself:
brute-force enumeration of what each reading says happens (every joint choice
of the other objects' trajectories, or every subset of independent
combinations), closed forms with one collision object, hand-computed ties, and
the identities the scaling must satisfy."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2005_06773_amd import scenegen as sg

EXCL, INDEP = oracle.RISK_EXCLUSIVE, oracle.RISK_INDEPENDENT


def veh(x, y, psi, v, u, w, L=4.5, W=1.8, score=None):
    return sg.SceneObject(sg.VEHICLE, x, y, psi, v, L, W, 0.0, np.asarray(u, float), np.asarray(w, float), score)


def ped(x, y, psi, v, u, w, r=0.3, score=None):
    return sg.SceneObject(sg.PEDESTRIAN, x, y, psi, v, 0.0, 0.0, r, np.asarray(u, float), np.asarray(w, float), score)


def random_tables(rng, T, H, ego_only=False, p_hit=0.5):
    """Random probabilities and first-hit tables (no geometry): the risk
    functions only see which combinations collide, and when."""
    n = len(T)
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n) if not ego_only or a == 0]
    p = np.concatenate([(lambda v: v / v.sum())(rng.uniform(0.05, 1.0, t)) for t in T])
    k = []
    for a, b in pairs:
        blk = rng.integers(0, H, T[a] * T[b])
        blk[rng.uniform(size=blk.size) > p_hit] = -1
        k.append(blk)
    k = np.concatenate(k).astype(np.int32)
    pa = np.array([a for a, _ in pairs], np.int32)
    pb = np.array([b for _, b in pairs], np.int32)
    return p, pa, pb, k


def combos_of(T, pa, pb, k, a, i):
    """(slot, b, j) of every colliding combination of trajectory (a, i)."""
    out = []
    e0 = 0
    for x, y in zip(pa.tolist(), pb.tolist()):
        blk = k[e0:e0 + T[x] * T[y]].reshape(T[x], T[y])
        if x == a:
            out += [(int(blk[i, j]), y, j) for j in range(T[y]) if blk[i, j] >= 0]
        elif y == a:
            out += [(int(blk[j, i]), x, j) for j in range(T[x]) if blk[j, i] >= 0]
        e0 += T[x] * T[y]
    return out


def brute_force(T, H, pa, pb, k, p, model):
    """Per trajectory: P(first collision at or before slot s) and P(first
    collision is with object b), by enumerating outcomes.
    EXCLUSIVE: every other object follows exactly one of its trajectories,
    independently of the others; INDEPENDENT: every colliding combination
    happens or not independently. Ties: ascending (slot, b, j)."""
    n = len(T)
    toff = np.concatenate([[0], np.cumsum(T)])
    ct = np.zeros((int(sum(T)), H))
    at = np.zeros((int(sum(T)), n))
    for a in range(n):
        for i in range(T[a]):
            ev = combos_of(T, pa, pb, k, a, i)
            row = toff[a] + i
            if model == EXCL:
                others = sorted({b for _, b, _ in ev})
                hit = {(b, j): s for s, b, j in ev}
                for choice in itertools.product(*[range(T[b]) for b in others]):
                    prob = 1.0
                    firsts = []
                    for b, j in zip(others, choice):
                        prob *= p[toff[b] + j]
                        if (b, j) in hit:
                            firsts.append((hit[(b, j)], b, j))
                    if firsts:
                        s0, b0, _ = min(firsts)
                        ct[row, s0:] += prob
                        at[row, b0] += prob
            else:
                for mask in range(1 << len(ev)):
                    prob = 1.0
                    happened = []
                    for e, (s, b, j) in enumerate(ev):
                        if mask >> e & 1:
                            prob *= p[toff[b] + j]
                            happened.append((s, b, j))
                        else:
                            prob *= 1.0 - p[toff[b] + j]
                    if happened:
                        s0, b0, _ = min(happened)
                        ct[row, s0:] += prob
                        at[row, b0] += prob
    return ct, at


@pytest.mark.parametrize("model", [EXCL, INDEP])
@pytest.mark.parametrize("seed", range(6))
def test_timeline_matches_brute_force(model, seed):
    rng = np.random.default_rng(100 + seed)
    T = [3, 2, 3, 2] if seed % 2 == 0 else [2, 3, 2]
    H = 5
    p, pa, pb, k = random_tables(rng, T, H, ego_only=(seed % 3 == 2))
    tct, oct_, tat, oat = oracle.risk_timeline_raw(T, H, pa, pb, k, p, model)
    ct, at = brute_force(T, H, pa, pb, k, p, model)
    assert np.allclose(tct, ct, atol=1e-13, rtol=0)
    assert np.allclose(tat, at, atol=1e-13, rtol=0)
    toff = np.concatenate([[0], np.cumsum(T)])
    for a in range(len(T)):
        w = p[toff[a]:toff[a + 1]]
        assert np.allclose(oct_[a], w @ ct[toff[a]:toff[a + 1]], atol=1e-13)
        assert np.allclose(oat[a], w @ at[toff[a]:toff[a + 1]], atol=1e-13)


@pytest.mark.parametrize("model", [EXCL, INDEP])
def test_whole_horizon_equals_risk_and_attribution_adds_up(model):
    """crit_t at the last slot is orc_risk's crit (1 - prod(1 - q)), the
    attribution over collision objects adds up to it, crit_t never decreases
    and nothing is attributed to an object itself or to a non-colliding one."""
    rng = np.random.default_rng(7)
    for trial in range(20):
        T = list(rng.integers(1, 6, rng.integers(2, 6)))
        H = int(rng.integers(1, 9))
        p, pa, pb, k = random_tables(rng, T, H, ego_only=bool(trial % 2), p_hit=rng.uniform(0.1, 0.9))
        tct, oct_, tat, oat = oracle.risk_timeline_raw(T, H, pa, pb, k, p, model)
        _, tc, oc = oracle.risk_raw(T, pa, pb, (k >= 0), p, model)
        assert np.allclose(tct[:, -1], tc, atol=1e-14)
        assert np.allclose(oct_[:, -1], oc, atol=1e-14)
        assert np.allclose(tat.sum(axis=1), tc, atol=1e-14)
        assert np.allclose(oat.sum(axis=1), oc, atol=1e-14)
        assert np.all(np.diff(tct, axis=1) >= -1e-15)
        assert np.all(tat >= 0) and np.all(np.diag(oat) == 0)
        n = len(T)
        for a in range(n):
            for b in range(n):
                if a != b and not any((x, y) in ((a, b), (b, a)) for x, y in zip(pa, pb)):
                    assert oat[a, b] == 0.0


def test_single_collision_object_closed_forms():
    """One collision object: EXCLUSIVE gives crit_t(s) = sum_j [k <= s] p_j
    (the paper's p_cra double sum, cut at s); INDEPENDENT gives
    1 - prod_{j: k <= s} (1 - p_j). All of it is attributed to that object."""
    rng = np.random.default_rng(11)
    T = [4, 5]
    H = 6
    p, pa, pb, k = random_tables(rng, T, H, p_hit=0.6)
    K = k.reshape(4, 5)
    pc = p[4:]
    for model in (EXCL, INDEP):
        tct, _, tat, _ = oracle.risk_timeline_raw(T, H, pa, pb, k, p, model)
        for i in range(4):
            for s in range(H):
                m = (K[i] >= 0) & (K[i] <= s)
                want = pc[m].sum() if model == EXCL else 1.0 - np.prod(1.0 - pc[m])
                assert tct[i, s] == pytest.approx(want, abs=1e-15)
            assert tat[i, 1] == pytest.approx(tct[i, -1], abs=1e-15) and tat[i, 0] == 0.0


def test_ties_go_to_the_lower_object_index():
    """By hand: the EGO's one trajectory meets CO 1 (p 0.5) and CO 2 (p 0.5)
    both at slot 2. Total 1 - 0.5 * 0.5 = 0.75 either way; CO 1 comes first
    (0.5), CO 2 keeps what CO 1 leaves (0.5 * 0.5). With CO 2 at slot 1 the
    roles swap."""
    T = [1, 2, 2]
    p = np.array([1.0, 0.5, 0.5, 0.5, 0.5])
    pa = np.array([0, 0], np.int32)
    pb = np.array([1, 2], np.int32)
    for model in (EXCL, INDEP):
        k = np.array([2, -1, 2, -1], np.int32)
        tct, _, tat, _ = oracle.risk_timeline_raw(T, 4, pa, pb, k, p, model)
        assert tct[0].tolist() == [0.0, 0.0, 0.75, 0.75]
        assert tat[0].tolist() == [0.0, 0.5, 0.25]
        k = np.array([3, -1, 1, -1], np.int32)
        tct, _, tat, _ = oracle.risk_timeline_raw(T, 4, pa, pb, k, p, model)
        assert tct[0].tolist() == [0.0, 0.5, 0.5, 0.75]
        assert tat[0].tolist() == [0.0, 0.25, 0.5]


def test_readings_differ_as_the_paper_allows():
    """Two colliding trajectories of one CO (p 0.5 each, slots 1 and 3):
    EXCLUSIVE adds them (crit 1.0: whichever the CO follows, it collides);
    INDEPENDENT gives 1 - 0.5 * 0.5 = 0.75, the paper's
    P(A) + P(~A) P(B). INDEPENDENT never exceeds EXCLUSIVE."""
    T = [1, 2]
    p = np.array([1.0, 0.5, 0.5])
    pa, pb = np.array([0], np.int32), np.array([1], np.int32)
    k = np.array([3, 1], np.int32)
    tct, _, _, _ = oracle.risk_timeline_raw(T, 4, pa, pb, k, p, EXCL)
    assert tct[0].tolist() == [0.0, 0.5, 0.5, 1.0]
    tct, _, _, _ = oracle.risk_timeline_raw(T, 4, pa, pb, k, p, INDEP)
    assert tct[0].tolist() == [0.0, 0.5, 0.5, 0.75]
    rng = np.random.default_rng(5)
    for _ in range(30):
        Tr = list(rng.integers(1, 7, 4))
        pr, pa2, pb2, k2 = random_tables(rng, Tr, 4)
        qe, tce, oce = oracle.risk_raw(Tr, pa2, pb2, k2 >= 0, pr, EXCL)
        qi, tci, oci = oracle.risk_raw(Tr, pa2, pb2, k2 >= 0, pr, INDEP)
        assert np.all(qi <= qe + 1e-15) and np.all(tci <= tce + 1e-15) and np.all(oci <= oce + 1e-15)


def test_head_on_timeline_is_a_step_at_the_closed_form_slot():
    """Deterministic head-on pair (one trajectory each): the criticality over
    time is 0 before slot n* - 1 and 1 from it on, n* = ceil((D - (L1+L2)/2) /
    ((v1+v2) tau)); every bit of it is attributed to the other vehicle."""
    rng = np.random.default_rng(9)
    done = 0
    while done < 20:
        D = rng.uniform(20, 60)
        v1, v2 = rng.uniform(2, 15, 2)
        tau = 0.1
        gap = (D - 4.5) / ((v1 + v2) * tau)
        if abs(gap - round(gap)) < 1e-6:
            continue
        H = int(math.ceil(gap)) + 4
        s = sg.Scene([veh(0, 0, 0, v1, [0.0], [0.0]), veh(D, 0, math.pi, v2, [0.0], [0.0])], H, tau, timeline=1)
        for model in (EXCL, INDEP):
            s.risk = model
            r = oracle.evaluate(s)
            step = np.zeros(H)
            step[int(math.ceil(gap)) - 1:] = 1.0
            assert np.array_equal(r.traj_crit_t[0], step) and np.array_equal(r.obj_crit_t[0], step)
            assert r.obj_attrib[0].tolist() == [0.0, 1.0] and r.obj_attrib[1].tolist() == [1.0, 0.0]
        done += 1


def _colliding_scene(seed, n=5, H=25):
    rng = np.random.default_rng(seed)
    objs = []
    for k in range(n):
        if k < 3:
            objs.append(veh(rng.uniform(-8, 8), rng.uniform(-8, 8), rng.uniform(0, 6.28), rng.uniform(2, 10),
                            sg.accel_grid(5), sg.yaw_grid(4), score=rng.uniform(0.1, 1.0, 20)))
        else:
            objs.append(ped(rng.uniform(-6, 6), rng.uniform(-6, 6), rng.uniform(0, 6.28), 1.0,
                            sg.ped_speed_grid(4), sg.ped_heading_grid(5), score=rng.uniform(0.1, 1.0, 20)))
    return sg.Scene(objs, H, 0.1, timeline=1)


@pytest.mark.parametrize("model", [EXCL, INDEP])
def test_scene_timeline_bounds_bracket_the_result(model):
    """On a geometric scene, the time-resolved bounds from the latest (lo) and
    earliest (hi) first hits the tolerance band allows bracket the value,
    and the last slot reproduces the plain criticality."""
    s = _colliding_scene(31)
    s.risk = model
    r = oracle.evaluate(s)
    assert r.obj_crit.max() > 0.05
    for mid, lo, hi in ((r.traj_crit_t, r.traj_crit_t_lo, r.traj_crit_t_hi),
                        (r.obj_crit_t, r.obj_crit_t_lo, r.obj_crit_t_hi)):
        assert np.all(lo <= mid + 1e-15) and np.all(mid <= hi + 1e-15)
    assert np.allclose(r.traj_crit_t[:, -1], r.traj_crit, atol=1e-14)
    assert np.allclose(r.obj_attrib.sum(axis=1), r.obj_crit, atol=1e-14)


def test_first_loose_slot_matches_the_masks():
    rng = np.random.default_rng(3)
    loose = np.zeros((200, 3), np.uint64)
    want = np.full(200, -1)
    for e in range(200):
        slots = sorted(rng.choice(150, rng.integers(0, 5), replace=False).tolist())
        for t in slots:
            loose[e, t // 64] |= np.uint64(1) << np.uint64(t % 64)
        if slots:
            want[e] = slots[0]
    assert np.array_equal(oracle.first_loose_slot(loose), want)
