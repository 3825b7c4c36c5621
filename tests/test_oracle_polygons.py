"""Pins of the oracle's general convex polygons (Sec. IV-C.1 allows object
polygons of any complexity).

The separating-axis margin is pinned by exact rational clipping (sign) and
closed forms (value); the polygon-circle margin by exact rational
point-polygon distances; the outline placement by the rectangle special case
and by a head-on closed form for pointed (diamond) outlines."""
import math

import numpy as np
import pytest

import oracle
from paper_2005_06773_amd import scenegen as sg
from tests import exact_geometry as eg


def place(outline, x, y, psi):
    """World vertices of a body-frame outline (numpy, not the oracle)."""
    c, s = math.cos(psi), math.sin(psi)
    o = np.asarray(outline, float)
    return np.stack([x + c * o[:, 0] - s * o[:, 1], y + s * o[:, 0] + c * o[:, 1]], axis=1)


def random_pair(rng, spread=6.0):
    P = place(sg.random_convex_outline(rng, int(rng.integers(3, 9)), rng.uniform(0.5, 2.0), rng.uniform(1, 2.5)),
              0.0, 0.0, rng.uniform(0, 2 * math.pi))
    Q = place(sg.random_convex_outline(rng, int(rng.integers(3, 9)), rng.uniform(0.5, 2.0), rng.uniform(1, 2.5)),
              rng.uniform(-spread, spread), rng.uniform(-spread, spread), rng.uniform(0, 2 * math.pi))
    return P, Q


def test_sat_sign_matches_exact_clipping():
    rng = np.random.default_rng(1)
    hits = misses = 0
    for _ in range(3000):
        P, Q = random_pair(rng)
        m = oracle.margin_poly_poly(P, Q)
        exact = eg.convex_intersect(eg.to_frac(P), eg.to_frac(Q))
        if abs(m) < 1e-12:
            continue
        assert (m <= 0) == exact
        hits += exact
        misses += not exact
    assert hits > 300 and misses > 300


def test_sat_closed_forms_and_invariances():
    sq = np.array([[1, -1], [1, 1], [-1, 1], [-1, -1]], float)   # 2 x 2 square, CCW
    for gap in (0.0, 0.37, 2.5, -0.4):
        Q = sq + [2.0 + gap, 0.3]
        assert oracle.margin_poly_poly(sq, Q) == pytest.approx(gap, abs=1e-14)
    # a diamond whose tip is g from the square's right side
    dia = np.array([[1.5, 0], [0, 1.5], [-1.5, 0], [0, -1.5]], float)
    for g in (0.2, 1.0):
        assert oracle.margin_poly_poly(sq, dia + [1.0 + 1.5 + g, 0.0]) == pytest.approx(g, abs=1e-14)
    rng = np.random.default_rng(2)
    for _ in range(300):
        P, Q = random_pair(rng)
        m = oracle.margin_poly_poly(P, Q)
        assert oracle.margin_poly_poly(Q, P) == pytest.approx(m, abs=1e-12)
        th = rng.uniform(0, 2 * math.pi)
        R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        t = rng.uniform(-50, 50, 2)
        assert oracle.margin_poly_poly(P @ R.T + t, Q @ R.T + t) == pytest.approx(m, abs=1e-9)
        # separated: moving Q further along the winning gap adds to the margin
        # no faster than the distance moved (1-Lipschitz)
        d = rng.uniform(-1, 1, 2)
        assert abs(oracle.margin_poly_poly(P, Q + d) - m) <= np.linalg.norm(d) + 1e-12


def test_rectangles_as_polygons_equal_the_rectangle_margin():
    rng = np.random.default_rng(3)
    for _ in range(500):
        A = (rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(0, 6.3), rng.uniform(3, 6), rng.uniform(1.5, 2.2))
        B = (rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(0, 6.3), rng.uniform(3, 6), rng.uniform(1.5, 2.2))
        P = eg.rect_corners_np(*A)
        Q = eg.rect_corners_np(*B)
        assert oracle.margin_poly_poly(P, Q) == pytest.approx(oracle.margin_rect_rect(A, B), abs=1e-12)


def test_poly_circle_against_exact_distance():
    rng = np.random.default_rng(4)
    inside = outside = 0
    for _ in range(2000):
        P = place(sg.random_convex_outline(rng, int(rng.integers(3, 9)), rng.uniform(0.5, 2), 1.7), 0, 0,
                  rng.uniform(0, 6.3))
        c = rng.uniform(-5, 5, 2)
        r = rng.uniform(0.1, 0.8)
        m = oracle.margin_poly_circle(P, c, r)
        d2 = eg.point_convex_dist2((eg.Fraction(float(c[0])), eg.Fraction(float(c[1]))), eg.to_frac(P))
        d = math.sqrt(float(d2))
        assert m == pytest.approx(d - r, abs=1e-12)
        if abs(m) > 1e-12:
            assert (m <= 0) == eg.rect_circle_intersect(eg.to_frac(P), (eg.Fraction(float(c[0])),
                                                                         eg.Fraction(float(c[1]))), r)
        inside += d2 == 0
        outside += d2 > 0
    assert inside > 50 and outside > 500


def test_pip_margin_on_outlines_is_the_vertex_test():
    """The point-in-polygon mode with outlines: hit iff some vertex of one lies
    in the other (exact rational half-plane containment)."""
    rng = np.random.default_rng(5)
    for _ in range(1500):
        P, Q = random_pair(rng, 4.0)
        m = oracle.margin_pip(P, Q)
        if abs(m) < 1e-12:
            continue
        fp, fq = eg.to_frac(P), eg.to_frac(Q)

        def inside(pt, poly):
            k = len(poly)
            return all(eg._cross(poly[e], poly[(e + 1) % k], pt) >= 0 for e in range(k))
        exact = any(inside(v, fq) for v in fp) or any(inside(v, fp) for v in fq)
        assert (m <= 0) == exact


def veh(x, y, psi, v, u, w, L=4.5, W=1.8, outline=None):
    return sg.SceneObject(sg.VEHICLE, x, y, psi, v, L, W, 0.0, np.asarray(u, float), np.asarray(w, float), None,
                          outline)


def test_outline_placement_matches_the_rectangle():
    """A vehicle whose outline is its own rectangle gives the same first hits
    as the rectangle, in both overlap modes."""
    s = sg.eleven_object_scene(2)
    s.objects = s.objects[:6]
    ref = oracle.evaluate(s, masks=False)
    for o in s.objects:
        l, w = o.length / 2, o.width / 2
        o.outline = np.array([[l, -w], [l, w], [-l, w], [-l, -w]])
    got = oracle.evaluate(s, masks=False)
    assert np.array_equal(ref.k64, got.k64)
    s.overlap = sg.OVERLAP_PIP
    for o in s.objects:
        o.outline = None
    ref = oracle.evaluate(s, masks=False)
    for o in s.objects:
        l, w = o.length / 2, o.width / 2
        o.outline = np.array([[l, -w], [l, w], [-l, w], [-l, -w]])
    assert np.array_equal(ref.k64, oracle.evaluate(s, masks=False).k64)


def test_one_outline_against_rectangles_matches_exact_clipping():
    """Only the EGO has an outline; the other vehicles are rectangles turned
    into polygons by the oracle. At sampled slots the oracle's first hits
    agree with exact rational clipping of the placed shapes."""
    from tests.exact_geometry import convex_intersect, to_frac, rect_corners_np
    s = sg.eleven_object_scene(6)
    s.objects = s.objects[:6]
    s.objects[0].outline = sg.car_outline(s.objects[0].length, s.objects[0].width, 0.5)
    r = oracle.evaluate(s, masks=False, threads=8)
    H, dt = s.horizon, s.dt
    T = s.traj_counts()
    xa, ya, pa = oracle.trajectories(s.objects[0], H, dt)
    rng = np.random.default_rng(7)
    checked = hits = 0
    for p, (a, b) in enumerate(zip(r.pair_a, r.pair_b)):
        if a != 0:
            continue
        xb, yb, pb = oracle.trajectories(s.objects[b], H, dt)
        blk = r.k64[r.pair_off[p]:r.pair_off[p + 1]].reshape(T[0], T[b])
        cand = list(zip(*np.nonzero(blk >= 0)))[:40] + [tuple(x) for x in rng.integers(0, [T[0], T[b]], (40, 2))]
        for i, j in cand:
            k = blk[i, j]
            slots = [k] if k >= 0 else []
            slots += [t for t in (0, H // 2, H - 1) if k < 0 or t < k]
            for t in slots:
                P = place(s.objects[0].outline, xa[t, i], ya[t, i], pa[t, i])
                Q = rect_corners_np(xb[t, j], yb[t, j], pb[t, j], s.objects[b].length, s.objects[b].width)
                m = oracle.margin_poly_poly(P, Q)
                if abs(m) > 1e-9:
                    assert convex_intersect(to_frac(P), to_frac(Q)) == (t == k), (a, b, i, j, t, k)
                    checked += 1
                    hits += t == k
    assert checked > 300 and hits > 20


def test_head_on_diamonds_closed_form():
    """Two diamond outlines (tips a1, a2 along the heading) driving at each
    other on one line touch tip to tip: n* = ceil((D - a1 - a2) / ((v1+v2) tau)),
    in both overlap modes (a tip is a vertex inside the other at contact)."""
    rng = np.random.default_rng(6)
    done = 0
    while done < 30:
        D = rng.uniform(20, 60)
        v1, v2 = rng.uniform(2, 15, 2)
        a1, a2 = rng.uniform(1.5, 3.0, 2)
        b1, b2 = rng.uniform(0.7, 1.2, 2)
        tau = 0.1
        gap = (D - a1 - a2) / ((v1 + v2) * tau)
        if abs(gap - round(gap)) < 1e-6:
            continue
        d1 = np.array([[a1, 0], [0, b1], [-a1, 0], [0, -b1]])
        d2 = np.array([[a2, 0], [0, b2], [-a2, 0], [0, -b2]])
        H = int(math.ceil(gap)) + 4
        s = sg.Scene([veh(0, 0, 0, v1, [0.0], [0.0], outline=d1), veh(D, 0, math.pi, v2, [0.0], [0.0], outline=d2)],
                     H, tau)
        assert oracle.evaluate(s, masks=False).k64[0] == math.ceil(gap) - 1
        done += 1


def test_octagon_cars_collide_no_earlier_than_their_rectangles():
    """The chamfered outline lies inside the rectangle, so every first hit of
    the octagon scene is at the same or a later slot (or none), and some
    differ."""
    s = sg.eleven_object_scene(9)
    rect = oracle.evaluate(s, masks=False, threads=8)
    poly = oracle.evaluate(sg.polygon_scene(9), masks=False, threads=8)
    kr = np.where(rect.k64 >= 0, rect.k64, 10 ** 6)
    kp = np.where(poly.k64 >= 0, poly.k64, 10 ** 6)
    assert np.all(kp >= kr)
    assert np.any(kp > kr)


def test_outline_rejected_for_pedestrians():
    s = sg.eleven_object_scene(0)
    s.objects = [s.objects[0], s.objects[7]]
    s.objects[1].outline = sg.car_outline(1.0, 1.0, 0.1)
    with pytest.raises(ValueError):
        oracle.evaluate(s)
