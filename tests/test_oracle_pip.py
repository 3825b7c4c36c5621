"""Pins of the oracle's point-in-polygon overlap mode (Sec. IV-C.1: the
vertices of each polygon are tested against the other polygon, both ways).

* closed forms: the plus sign (a miss, margin 1.35 m), containment, a shared
  corner (margin 0, a hit), separated squares;
* exact rational geometry on random rectangles and convex polygons: the
  sign of the margin against half-plane vertex containment, its magnitude
  against exact squared distances to the other polygon's edges;
* a point-in-polygon hit is always an overlap, so first hits in this mode
  are never earlier than exact ones; two crossings with hand-computed steps;
* the mode takes rectangles only.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2005_06773_amd import scenegen as sg
from tests import exact_geometry as eg


def _rand_rect(rng, spread):
    return (rng.uniform(-spread, spread), rng.uniform(-spread, spread), rng.uniform(0, 2 * math.pi),
            rng.uniform(0.5, 5.0), rng.uniform(0.3, 2.5))


def _rand_convex(rng, spread, n):
    """Convex polygon: n sorted angles on an ellipse, rotated and shifted."""
    ang = np.sort(rng.uniform(0, 2 * math.pi, n))
    a, b = rng.uniform(0.5, 3.0), rng.uniform(0.3, 2.0)
    rot = rng.uniform(0, 2 * math.pi)
    x, y = a * np.cos(ang), b * np.sin(ang)
    c, s = math.cos(rot), math.sin(rot)
    return np.stack([c * x - s * y + rng.uniform(-spread, spread), s * x + c * y + rng.uniform(-spread, spread)], 1)


def _inside_closed(p, poly):
    poly = eg._ccw(poly)
    n = len(poly)
    return all(eg._cross(poly[k], poly[(k + 1) % n], p) >= 0 for k in range(n))


def _exact_pip_margin(P, Q):
    """min over the vertices of both polygons of the signed distance to the
    other polygon's boundary, from exact rationals (sqrt taken at the end)."""
    best = None
    for A, B in ((P, Q), (Q, P)):
        for v in A:
            d2 = min(eg.point_segment_dist2(v, B[k], B[(k + 1) % len(B)]) for k in range(len(B)))
            s = -math.sqrt(d2) if _inside_closed(v, B) else math.sqrt(d2)
            best = s if best is None else min(best, s)
    return best


def test_closed_forms():
    # plus sign: every corner 2.25 - 0.9 = 1.35 m outside the other bar
    assert oracle.margin_rect_rect_pip((0, 0, 0, 4.5, 1.8), (0, 0, math.pi / 2, 4.5, 1.8)) == pytest.approx(1.35, abs=1e-12)
    assert oracle.margin_rect_rect((0, 0, 0, 4.5, 1.8), (0, 0, math.pi / 2, 4.5, 1.8)) < 0
    # a 1 x 1 square inside a 4 x 2 rectangle: its corners are 0.5 m deep
    assert oracle.margin_rect_rect_pip((0, 0, 0, 4, 2), (0, 0, 0, 1, 1)) == pytest.approx(-0.5, abs=1e-12)
    # shared corner (2, 1): touching counts
    assert oracle.margin_rect_rect_pip((0, 0, 0, 4, 2), (2.5, 1.5, 0, 1, 1)) == pytest.approx(0.0, abs=1e-12)
    # 2 x 2 squares 5 m apart: the nearest corner is 3 m from the other square
    assert oracle.margin_rect_rect_pip((0, 0, 0, 2, 2), (5, 0, 0, 2, 2)) == pytest.approx(3.0, abs=1e-12)


def test_rectangle_wrapper_is_the_polygon_margin():
    rng = np.random.default_rng(31)
    for _ in range(500):
        P, Q = _rand_rect(rng, 1.0), _rand_rect(rng, 3.0)
        m_poly = oracle.margin_pip(oracle.rect_corners(*P), oracle.rect_corners(*Q))
        assert oracle.margin_rect_rect_pip(P, Q) == m_poly


@pytest.mark.parametrize("shape", ["rect", "convex"])
def test_sign_and_magnitude_vs_exact(shape):
    rng = np.random.default_rng(2024 if shape == "rect" else 2025)
    n_hit = n_miss = 0
    for _ in range(1500):
        if shape == "rect":
            cp, cq = eg.rect_corners_np(*_rand_rect(rng, 0.5)), eg.rect_corners_np(*_rand_rect(rng, 4.0))
        else:
            cp, cq = _rand_convex(rng, 0.5, int(rng.integers(3, 8))), _rand_convex(rng, 4.0, int(rng.integers(3, 8)))
        m = oracle.margin_pip(cp, cq)
        P, Q = eg.to_frac(cp), eg.to_frac(cq)
        ex = _exact_pip_margin(P, Q)
        assert m == pytest.approx(ex, abs=1e-9), (cp, cq)
        if abs(m) > 1e-9:
            hit = any(_inside_closed(v, Q) for v in P) or any(_inside_closed(v, P) for v in Q)
            assert hit == (m <= 0)
            n_hit += hit
            n_miss += not hit
    assert n_hit > 200 and n_miss > 200


def test_pip_hit_implies_exact_overlap():
    rng = np.random.default_rng(77)
    n = 0
    for _ in range(4000):
        P, Q = _rand_rect(rng, 0.5), _rand_rect(rng, 3.0)
        if oracle.margin_rect_rect_pip(P, Q) <= 0:
            n += 1
            assert oracle.margin_rect_rect(P, Q) <= 1e-12
    assert n > 500


def _veh(x, y, psi, v, L=4.5, W=1.8):
    return sg.SceneObject(sg.VEHICLE, x, y, psi, v, L, W, 0.0, np.array([0.0]), np.array([0.0]), None)


def _both_modes(objs, H, dt):
    ex = oracle.evaluate(sg.Scene(objs, H, dt), masks=False, risk=False)
    pip = oracle.evaluate(sg.Scene(objs, H, dt, overlap=sg.OVERLAP_PIP), masks=False, risk=False)
    return ex.k64, pip.k64


def test_plus_sign_crossing_missed_in_pip_mode():
    """A drives through a perpendicular, stationary B at 10 m/s with 1 s
    steps: at step 1 it sits exactly on B's centre (a plus sign), at step 2
    it has passed. The exact test hits at slot 0, the paper's test never."""
    k_ex, k_pip = _both_modes([_veh(-10, 0, 0.0, 10.0), _veh(0, 0, math.pi / 2, 0.0)], 2, 1.0)
    assert k_ex.tolist() == [0] and k_pip.tolist() == [-1]


def test_t_bone_first_step_in_both_modes():
    """A (4.5 x 1.8 m) approaches a perpendicular B from x = -10 m at 10 m/s,
    20 ms steps. A's front corners enter B's side when
    -10 + 0.2 n + 2.25 >= -0.9, first at n = 35 (slot 34), in both modes."""
    k_ex, k_pip = _both_modes([_veh(-10, 0, 0.0, 10.0), _veh(0, 0, math.pi / 2, 0.0)], 60, 0.02)
    assert k_ex.tolist() == [34] and k_pip.tolist() == [34]


def test_first_hits_never_earlier_than_exact():
    """On paper-like scenes with coarse 0.1 s steps, where the two modes do
    differ, every point-in-polygon first hit is also an exact hit, and the
    exact first hit comes at the same step or earlier."""
    total = differ = 0
    for seed in range(4):
        s = sg.paper_scene(seed, n_co=4, n_acc=2)
        s.dt, s.horizon = 0.1, 30
        s.objects[0].w = s.objects[0].w[::49]
        s.objects[0].score = None
        k_ex = oracle.evaluate(s, masks=False, risk=False).k64
        s.overlap = sg.OVERLAP_PIP
        k_pip = oracle.evaluate(s, masks=False, risk=False).k64
        both = k_pip >= 0
        assert np.all(k_ex[both] >= 0) and np.all(k_pip[both] >= k_ex[both])
        total += int((k_ex >= 0).sum())
        differ += int((k_pip != k_ex).sum())
    assert total > 20 and differ > 0, (total, differ)


def test_pip_mode_takes_rectangles_only():
    s = sg.Scene([_veh(0, 0, 0, 1), sg.SceneObject(sg.PEDESTRIAN, 3, 0, 0, 1, 0, 0, 0.3, np.array([1.0]), np.array([0.0]))],
                 5, 0.1, overlap=sg.OVERLAP_PIP)
    with pytest.raises(ValueError):
        oracle.evaluate(s, masks=False, risk=False)
