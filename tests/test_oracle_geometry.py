"""Pins of the oracle's overlap margins (Sec. IV-C.1) against exact geometry.

* exact rational convex clipping / exact squared distances on random tiny
  pose pairs (brute force, agreement wherever |m| > 1e-9);
* closed forms: axis-aligned rectangles, circles;
* the paper's point-in-polygon test run both ways implies overlap, and the
  "plus sign" shows why it is not used as the definition;
* the tunnelling thresholds printed in Sec. IV-C.2.
"""
import math

import numpy as np
import pytest

import oracle
from tests import exact_geometry as eg


def _rand_rect(rng, spread):
    return (rng.uniform(-spread, spread), rng.uniform(-spread, spread), rng.uniform(0, 2 * math.pi),
            rng.uniform(0.5, 5.0), rng.uniform(0.3, 2.5))


def test_rect_rect_sign_vs_exact_clipping():
    rng = np.random.default_rng(12345)
    n_hit = n_miss = 0
    for _ in range(6000):
        P = _rand_rect(rng, 0.5)
        Q = _rand_rect(rng, 4.0)
        m = oracle.margin_rect_rect(P, Q)
        if abs(m) <= 1e-9:
            continue
        ex = eg.convex_intersect(eg.to_frac(eg.rect_corners_np(*P)), eg.to_frac(eg.rect_corners_np(*Q)))
        assert ex == (m <= 0), (P, Q, m)
        n_hit += ex
        n_miss += not ex
    assert n_hit > 1000 and n_miss > 1000


def test_rect_circle_sign_vs_exact_distance():
    rng = np.random.default_rng(777)
    n_hit = n_miss = 0
    for _ in range(6000):
        P = _rand_rect(rng, 0.5)
        cx, cy, r = rng.uniform(-4, 4), rng.uniform(-4, 4), rng.uniform(0.05, 1.5)
        m = oracle.margin_rect_circle(P, (cx, cy, r))
        if abs(m) <= 1e-9:
            continue
        ex = eg.rect_circle_intersect(eg.to_frac(eg.rect_corners_np(*P)),
                                      eg.to_frac(np.array([[cx, cy]]))[0], r)
        assert ex == (m <= 0), (P, cx, cy, r, m)
        n_hit += ex
        n_miss += not ex
    assert n_hit > 500 and n_miss > 500


def test_rect_circle_margin_is_euclidean_distance():
    """Outside the rectangle the margin is the exact distance minus r."""
    rng = np.random.default_rng(4242)
    for _ in range(2000):
        P = _rand_rect(rng, 0.5)
        cx, cy, r = rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(0.05, 1.5)
        m = oracle.margin_rect_circle(P, (cx, cy, r))
        d2 = eg.point_convex_dist2(eg.to_frac(np.array([[cx, cy]]))[0], eg.to_frac(eg.rect_corners_np(*P)))
        d = math.sqrt(float(d2))
        assert abs((m + r) - d) < 1e-9


def test_circle_circle_sign_and_value():
    rng = np.random.default_rng(99)
    for _ in range(4000):
        a = (rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.05, 1.0))
        b = (rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.05, 1.0))
        m = oracle.margin_circle_circle(a, b)
        if abs(m) > 1e-9:
            ex = eg.circle_circle_intersect((eg.Fraction(a[0]), eg.Fraction(a[1])), a[2],
                                            (eg.Fraction(b[0]), eg.Fraction(b[1])), b[2])
            assert ex == (m <= 0)
        assert abs(m - (math.dist(a[:2], b[:2]) - a[2] - b[2])) < 1e-12


def test_axis_aligned_rectangles_closed_form():
    """With both headings 0 the rectangles are boxes: the margin is the larger
    of the two interval gaps."""
    rng = np.random.default_rng(5)
    for _ in range(2000):
        LP, WP, LQ, WQ = rng.uniform(0.5, 5, 4)
        dx, dy = rng.uniform(-6, 6, 2)
        m = oracle.margin_rect_rect((0, 0, 0, LP, WP), (dx, dy, 0, LQ, WQ))
        expect = max(abs(dx) - (LP + LQ) / 2, abs(dy) - (WP + WQ) / 2)
        assert abs(m - expect) < 1e-12
        # rotating both boxes by the same angle about the origin changes nothing
        th = rng.uniform(0, 2 * math.pi)
        c, s = math.cos(th), math.sin(th)
        m2 = oracle.margin_rect_rect((0, 0, th, LP, WP), (c * dx - s * dy, s * dx + c * dy, th, LQ, WQ))
        assert abs(m2 - expect) < 1e-9


def test_margin_symmetric_in_arguments():
    rng = np.random.default_rng(6)
    for _ in range(1000):
        P, Q = _rand_rect(rng, 1.0), _rand_rect(rng, 3.0)
        assert oracle.margin_rect_rect(P, Q) == pytest.approx(oracle.margin_rect_rect(Q, P), abs=1e-12)


def test_point_in_polygon_both_ways_implies_overlap():
    """Sec. IV-C.1 tests each polygon's vertices against the other; whenever
    that reports a collision the rectangles do overlap."""
    rng = np.random.default_rng(11)
    n_pip = 0
    for _ in range(3000):
        P, Q = _rand_rect(rng, 0.5), _rand_rect(rng, 3.0)
        cp = oracle.rect_corners(*P)
        cq = oracle.rect_corners(*Q)
        pip = any(oracle.point_in_polygon(x, y, cq) for x, y in cp) or \
            any(oracle.point_in_polygon(x, y, cp) for x, y in cq)
        if pip:
            n_pip += 1
            assert oracle.margin_rect_rect(P, Q) <= 0
    assert n_pip > 300


def test_plus_sign_overlap_missed_by_point_in_polygon():
    """Two 4.5 x 1.8 m rectangles on one centre crossed at 90 degrees overlap,
    yet no vertex of either lies inside the other."""
    P = (0.0, 0.0, 0.0, 4.5, 1.8)
    Q = (0.0, 0.0, math.pi / 2, 4.5, 1.8)
    cp, cq = oracle.rect_corners(*P), oracle.rect_corners(*Q)
    assert not any(oracle.point_in_polygon(x, y, cq) for x, y in cp)
    assert not any(oracle.point_in_polygon(x, y, cp) for x, y in cq)
    assert oracle.margin_rect_rect(P, Q) < -0.5


def _read_golden():
    import os
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, val = line.split()[:2]
            vals[name] = int(val)
    return vals


def _tunnel_missed(speed, orientation_b, phases=400):
    """Car A (3.13 x 1.46 m) drives along x through stationary car B at
    constant ``speed`` with 20 ms steps; returns True if some start phase lets
    A jump over B without any colliding step (oracle first hit -1)."""
    from paper_2005_06773_amd import scenegen as sg
    tau = 0.02
    step = speed * tau
    for k in range(phases):
        x0 = -30.0 - step * (k + 0.5) / phases
        H = int(60.0 / step) + 2
        A = sg.SceneObject(sg.VEHICLE, x0, 0.0, 0.0, speed, 3.13, 1.46, 0.0,
                           np.array([0.0]), np.array([0.0]), None)
        B = sg.SceneObject(sg.VEHICLE, 0.0, 0.0, orientation_b, 0.0, 3.13, 1.46, 0.0,
                           np.array([0.0]), np.array([0.0]), None)
        r = oracle.evaluate(sg.Scene([A, B], H, tau), masks=False, risk=False)
        if r.k64[0] < 0:
            return True
    return False


def test_tunnelling_thresholds_of_the_paper():
    """Sec. IV-C.2: at 20 ms a T-bone needs 229 m/s and a longitudinal pass
    313 m/s of relative speed to go through undetected. The exact thresholds
    are (L+W)/tau = 229.5 m/s and 2L/tau = 313 m/s."""
    g = _read_golden()
    tb, lo = g["tunnel_tbone_mps"], g["tunnel_longitudinal_mps"]
    assert not _tunnel_missed(tb, math.pi / 2)          # 229 m/s: always caught
    assert _tunnel_missed(tb + 1, math.pi / 2)          # 230 m/s: some phase slips
    assert not _tunnel_missed(lo - 1, 0.0)              # 312 m/s: always caught
    assert _tunnel_missed(lo + 1, 0.0)                  # 314 m/s: some phase slips
