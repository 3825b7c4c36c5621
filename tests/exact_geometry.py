"""Exact rational geometry used to pin the oracle's overlap margins.

Shapes are given by FP64 corner coordinates (computed here with numpy, not by
the oracle) which are converted to ``fractions.Fraction`` exactly; every
decision below is then exact. Nothing here is shared with the oracle or the
GPU library.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Tuple

import numpy as np

Pt = Tuple[Fraction, Fraction]


def rect_corners_np(x, y, psi, L, W) -> np.ndarray:
    """Counter-clockwise corners of a rectangle (numpy FP64)."""
    u = np.array([np.cos(psi), np.sin(psi)])
    v = np.array([-np.sin(psi), np.cos(psi)])
    c = np.array([x, y])
    hl, hw = L / 2.0, W / 2.0
    return np.array([c + hl * u + hw * v, c - hl * u + hw * v, c - hl * u - hw * v, c + hl * u - hw * v])


def to_frac(poly: np.ndarray) -> List[Pt]:
    return [(Fraction(float(px)), Fraction(float(py))) for px, py in poly]


def _cross(o: Pt, a: Pt, b: Pt) -> Fraction:
    return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])


def _ccw(poly: List[Pt]) -> List[Pt]:
    area = sum(poly[k][0] * poly[(k + 1) % len(poly)][1] - poly[(k + 1) % len(poly)][0] * poly[k][1]
               for k in range(len(poly)))
    return poly if area >= 0 else poly[::-1]


def clip_convex(subject: List[Pt], clip: List[Pt]) -> List[Pt]:
    """Sutherland-Hodgman clipping of ``subject`` by the closed convex polygon
    ``clip``. Exact in rationals; a touching contact leaves a degenerate
    (point or segment) result, which still counts as an intersection."""
    out = list(subject)
    clip = _ccw(clip)
    n = len(clip)
    for k in range(n):
        a, b = clip[k], clip[(k + 1) % n]
        inp = out
        out = []
        if not inp:
            break
        for m in range(len(inp)):
            cur, prev = inp[m], inp[m - 1]
            dc, dp = _cross(a, b, cur), _cross(a, b, prev)
            if dc >= 0:
                if dp < 0:
                    out.append(_intersect(prev, cur, dp, dc))
                out.append(cur)
            elif dp >= 0:
                out.append(_intersect(prev, cur, dp, dc))
    return out


def _intersect(p: Pt, c: Pt, dp: Fraction, dc: Fraction) -> Pt:
    t = dp / (dp - dc)
    return (p[0] + t * (c[0] - p[0]), p[1] + t * (c[1] - p[1]))


def convex_intersect(P: List[Pt], Q: List[Pt]) -> bool:
    return len(clip_convex(P, Q)) > 0


def point_segment_dist2(p: Pt, a: Pt, b: Pt) -> Fraction:
    dx, dy = b[0] - a[0], b[1] - a[1]
    L2 = dx * dx + dy * dy
    if L2 == 0:
        t = Fraction(0)
    else:
        t = ((p[0] - a[0]) * dx + (p[1] - a[1]) * dy) / L2
        t = min(max(t, Fraction(0)), Fraction(1))
    cx, cy = a[0] + t * dx - p[0], a[1] + t * dy - p[1]
    return cx * cx + cy * cy


def point_convex_dist2(p: Pt, poly: List[Pt]) -> Fraction:
    poly = _ccw(poly)
    n = len(poly)
    inside = all(_cross(poly[k], poly[(k + 1) % n], p) >= 0 for k in range(n))
    if inside:
        return Fraction(0)
    return min(point_segment_dist2(p, poly[k], poly[(k + 1) % n]) for k in range(n))


def rect_circle_intersect(rect: List[Pt], c: Pt, r: float) -> bool:
    rr = Fraction(float(r))
    return point_convex_dist2(c, rect) <= rr * rr


def circle_circle_intersect(c1: Pt, r1: float, c2: Pt, r2: float) -> bool:
    s = Fraction(float(r1)) + Fraction(float(r2))
    dx, dy = c2[0] - c1[0], c2[1] - c1[1]
    return dx * dx + dy * dy <= s * s
