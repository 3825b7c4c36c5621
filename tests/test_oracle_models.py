"""Pins of the oracle's other motion models (Sec. IV-B.1 one-track model for
vehicles, Sec. IV-B.3 pedestrian acceleration model with its 2.7 m/s cap).

Pedestrians: closed forms for cruising, reaching the cap and stopping.
One-track model: a straight line without steering (the constant-acceleration
closed form), the textbook steady-state yaw rate of the linear one-track
model (understeer gradient) reached at speed, mirror symmetry, rest, the
low-speed steady state, and the understeer ordering by mass."""
import math

import numpy as np
import pytest

import oracle
from paper_2005_06773_amd import scenegen as sg


def ped(x, y, v, accels, headings, v_max=2.7, psi=0.3):
    return sg.SceneObject(sg.PEDESTRIAN, x, y, psi, v, 0.0, 0.0, 0.3, np.asarray(accels, float),
                          np.asarray(headings, float), None, None, sg.MODEL_PED_ACCEL, np.array([v_max]))


def ot(v, accels, steer, params=None, psi=0.0, x=0.0, y=0.0):
    p = sg.one_track_params(4.5) if params is None else np.asarray(params, float)
    return sg.SceneObject(sg.VEHICLE, x, y, psi, v, 4.5, 1.8, 0.0, np.asarray(accels, float),
                          np.asarray(steer, float), None, None, sg.MODEL_ONE_TRACK, p)


def test_pedestrian_cruise_along_absolute_heading():
    """a = 0: x_n = x0 + n tau v0 cos(h), whatever the measured heading."""
    for h in (0.0, 1.1, 3.5):
        o = ped(1.0, -2.0, 1.4, [0.0], [h], psi=2.0)
        x, y, psi = oracle.trajectories(o, 20, 0.1)
        n = np.arange(1, 21)
        assert np.allclose(x[:, 0], 1.0 + n * 0.1 * 1.4 * math.cos(h), atol=1e-12)
        assert np.allclose(y[:, 0], -2.0 + n * 0.1 * 1.4 * math.sin(h), atol=1e-12)
        assert np.all(psi[:, 0] == h)


def test_pedestrian_reaches_the_cap_and_stays():
    """v0 = 1, a = 2, tau = 0.1, cap 2.7: the speed after n steps is
    min(1 + 0.2 n, 2.7); each step advances by the mean of its two speeds."""
    o = ped(0.0, 0.0, 1.0, [2.0], [0.0])
    x, _, _ = oracle.trajectories(o, 30, 0.1)
    v = np.minimum(1.0 + 0.2 * np.arange(31), 2.7)
    want = np.cumsum((v[:-1] + v[1:]) / 2 * 0.1)
    assert np.allclose(x[:, 0], want, atol=1e-12)
    assert x[-1, 0] - x[-2, 0] == pytest.approx(0.27, abs=1e-12)


def test_pedestrian_stops():
    """a = -12 from 2 m/s at tau = 0.05: full steps while v > |a| tau, then
    the cut step; distance (v0^2 - v_k^2) / (2|a|) + v_k tau / 2."""
    o = ped(0.0, 0.0, 2.0, [-12.0], [0.0])
    x, _, _ = oracle.trajectories(o, 10, 0.05)
    k = int(2.0 // 0.6)                   # full steps of 0.6 m/s
    vk = 2.0 - 0.6 * k
    assert x[-1, 0] == pytest.approx((4.0 - vk ** 2) / 24.0 + vk * 0.05 / 2, abs=1e-12)
    assert x[-1, 0] == x[-3, 0]


def test_one_track_without_steering_is_the_straight_line():
    for v0, a in ((12.0, 0.0), (8.0, 1.5), (15.0, -3.0)):
        o = ot(v0, [a], [0.0], psi=0.7)
        x, y, psi = oracle.trajectories(o, 40, 0.05)
        t = np.arange(1, 41) * 0.05
        s = v0 * t + a * t * t / 2
        assert np.allclose(x[:, 0], s * math.cos(0.7), atol=1e-10)
        assert np.allclose(y[:, 0], s * math.sin(0.7), atol=1e-10)
        assert np.allclose(psi[:, 0], 0.7, atol=1e-15)


def _steady_yaw_rate(p, v, delta):
    """Textbook linear one-track steady state: r = v delta / (L (1 + K v^2)),
    K = m (lr cr - lf cf) / (L^2 cf cr)."""
    cf, cr, lf, lr, m, _ = p
    L = lf + lr
    K = m * (lr * cr - lf * cf) / (L * L * cf * cr)
    return v * delta / (L * (1 + K * v * v))


@pytest.mark.parametrize("v,delta", [(20.0, 0.03), (30.0, -0.02), (12.0, 0.06)])
def test_one_track_settles_to_the_textbook_yaw_rate_and_circle(v, delta):
    p = sg.one_track_params(4.5)
    tau = 0.005
    H = 2000
    x, y, psi = oracle.trajectories(ot(v, [0.0], [delta], params=p), H, tau)
    r = _steady_yaw_rate(p, v, delta)
    rate = (psi[-1, 0] - psi[-2, 0]) / tau
    assert rate == pytest.approx(r, rel=1e-9)
    # the path is a circle of radius v / r: curvature from three late points
    P = np.stack([x[-400:, 0], y[-400:, 0]], axis=1)[::100]
    a, b, c = P[0], P[1], P[2]
    area2 = abs((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))
    R = np.linalg.norm(a - b) * np.linalg.norm(b - c) * np.linalg.norm(c - a) / (2 * area2)
    assert R == pytest.approx(v / abs(r), rel=2e-3)


def test_one_track_mirror_symmetry_and_rest():
    p = sg.one_track_params(4.2)
    o = ot(9.0, [-2.0, 1.0], [-0.05, 0.05], params=p)
    x, y, psi = oracle.trajectories(o, 60, 0.1)
    for k in range(2):
        assert np.allclose(x[:, 2 * k], x[:, 2 * k + 1], atol=1e-12)
        assert np.allclose(y[:, 2 * k], -y[:, 2 * k + 1], atol=1e-12)
        assert np.allclose(psi[:, 2 * k], -psi[:, 2 * k + 1], atol=1e-12)
    x, y, psi = oracle.trajectories(ot(0.0, [0.0, -3.0], [0.08], params=p, x=3.0, y=4.0, psi=1.0), 30, 0.1)
    assert np.all(x == 3.0) and np.all(y == 4.0) and np.all(psi == 1.0)


def test_one_track_low_speed_takes_the_steady_state():
    """At 2 m/s and 0.1 s steps the Euler step is unstable, so every step
    takes the steady state: the heading advances by the mean of the steady
    yaw rates before and after (the first step from r = 0)."""
    p = sg.one_track_params(4.5)
    v, delta, tau = 2.0, 0.08, 0.1
    x, y, psi = oracle.trajectories(ot(v, [0.0], [delta], params=p), 20, tau)
    r = _steady_yaw_rate(p, v, delta)
    steps = np.diff(np.concatenate([[0.0], psi[:, 0]]))
    assert steps[0] == pytest.approx(r * tau / 2, rel=1e-12)
    assert np.allclose(steps[1:], r * tau, rtol=1e-12)
    # from the second step on, beta and r are constant (textbook steady
    # state) and the speed too, so a_x = -sin(beta) v r, a_y = cos(beta) v r
    # and each step moves by v tau R(psi_n) [(cos b, sin b) + (tau r / 2)(-sin b, cos b)]
    cf, cr, lf, lr, m, _ = p
    L = lf + lr
    K = m * (lr * cr - lf * cf) / (L * L * cf * cr)
    b = delta * (lr / L - m * lf * v * v / (cr * L * L)) / (1 + K * v * v)
    for n in range(1, 19):
        ps = psi[n, 0]
        local = np.array([math.cos(b) - tau * r / 2 * math.sin(b), math.sin(b) + tau * r / 2 * math.cos(b)])
        want = v * tau * np.array([math.cos(ps) * local[0] - math.sin(ps) * local[1],
                                   math.sin(ps) * local[0] + math.cos(ps) * local[1]])
        got = np.array([x[n + 1, 0] - x[n, 0], y[n + 1, 0] - y[n, 0]])
        assert np.allclose(got, want, atol=1e-13)


def test_heavier_vehicle_turns_less():
    """Understeer: with everything else equal, more mass means a larger
    understeer gradient and a smaller yaw rate at speed."""
    p = sg.one_track_params(4.5)
    q = p.copy()
    q[4] *= 1.5
    rates = []
    for par in (p, q):
        _, _, psi = oracle.trajectories(ot(25.0, [0.0], [0.02], params=par), 3000, 0.005)
        rates.append((psi[-1, 0] - psi[-2, 0]) / 0.005)
    assert rates[1] < rates[0]
    assert rates[1] == pytest.approx(_steady_yaw_rate(q, 25.0, 0.02), rel=1e-9)


def test_models_rejected_where_they_do_not_apply():
    o = ped(0, 0, 1, [0.0], [0.0])
    o.kind = sg.VEHICLE
    with pytest.raises(ValueError):
        oracle.trajectories(o, 5, 0.1)
    p = sg.one_track_params(4.5)
    p[2], p[3] = 2.0, 0.5       # oversteer
    with pytest.raises(ValueError):
        oracle.trajectories(ot(10.0, [0.0], [0.0], params=p), 5, 0.1)
