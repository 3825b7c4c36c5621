"""The DPP moves of the trajectory kernel's wave scans (kernels.hip,
scan_add and the one-track composition), simulated lane by lane: shifts by
1, 2, 4 and 8 lanes within each row of 16 lanes (a lane without a source in
its row gets the identity), then lane 15 of rows 0 and 2 into rows 1 and 3,
then lane 31 into rows 2 and 3. After the six steps every lane must hold
the combination of lanes 0..l in lane order: for sums, and for an
order-sensitive combination (the composition of affine maps does not
commute), here concatenation of lane sequences."""
import random


def _row_shr(v, n, identity):
    return [v[l - n] if l - n >= 0 and (l - n) // 16 == l // 16 else identity for l in range(64)]


def _row_bcast15(v, identity):  # row mask 0xA: rows 1 and 3 take lane 15 of the row below
    return [v[(l // 16) * 16 - 1] if l // 16 in (1, 3) else identity for l in range(64)]


def _row_bcast31(v, identity):  # row mask 0xC: rows 2 and 3 take lane 31
    return [v[31] if l // 16 in (2, 3) else identity for l in range(64)]


def _wave_scan(x, combine, identity):
    v = list(x)
    for n in (1, 2, 4, 8):
        v = [combine(t, m) for m, t in zip(v, _row_shr(v, n, identity))]
    v = [combine(t, m) for m, t in zip(v, _row_bcast15(v, identity))]
    v = [combine(t, m) for m, t in zip(v, _row_bcast31(v, identity))]
    return v


def test_sum_scan_is_the_inclusive_prefix():
    rng = random.Random(7)
    x = [rng.randint(-1000, 1000) for _ in range(64)]
    assert _wave_scan(x, lambda earlier, mine: earlier + mine, 0) == [sum(x[:l + 1]) for l in range(64)]


def test_ordered_scan_keeps_lane_order():
    # (earlier lanes) then (this lane's part): the map of lane l becomes
    # f_l o ... o f_0, as the one-track model composes them
    got = _wave_scan([(l,) for l in range(64)], lambda earlier, mine: earlier + mine, ())
    assert got == [tuple(range(l + 1)) for l in range(64)]


def test_affine_maps_compose_in_lane_order():
    rng = random.Random(11)
    maps = [((rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-1, 1)),
             (rng.uniform(-1, 1), rng.uniform(-1, 1))) for _ in range(64)]

    def compose(earlier, mine):  # mine o earlier: (A, b) o (P, q) = (AP, Aq + b)
        (a11, a12, a21, a22), (b1, b2) = mine
        (p11, p12, p21, p22), (q1, q2) = earlier
        return ((a11 * p11 + a12 * p21, a11 * p12 + a12 * p22, a21 * p11 + a22 * p21, a21 * p12 + a22 * p22),
                (a11 * q1 + a12 * q2 + b1, a21 * q1 + a22 * q2 + b2))
    identity = ((1.0, 0.0, 0.0, 1.0), (0.0, 0.0))
    got = _wave_scan(maps, compose, identity)
    s = (0.3, -0.7)
    for l in (0, 1, 15, 16, 17, 31, 32, 47, 48, 63):
        want = s
        for k in range(l + 1):   # apply f_0, then f_1, ... f_l
            (a11, a12, a21, a22), (b1, b2) = maps[k]
            want = (a11 * want[0] + a12 * want[1] + b1, a21 * want[0] + a22 * want[1] + b2)
        (a11, a12, a21, a22), (b1, b2) = got[l]
        z = (a11 * s[0] + a12 * s[1] + b1, a21 * s[0] + a22 * s[1] + b2)
        assert abs(z[0] - want[0]) < 1e-9 and abs(z[1] - want[1]) < 1e-9, l
