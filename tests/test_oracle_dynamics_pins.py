"""Pins of the oracle's model means by properties their physics fixes.

The unicycle (the 3-D reach-avoid workload), the room ring (Sec. 8.2) and
the 7-D single-track vehicle (Sec. 8.4.1) are model definitions, so no
printed value exists to compare the oracle's mean mu = f(x, u) with.  Each
test below checks a property that follows from what the model describes:
geometry of motion, equilibria, locality and symmetry of heat conduction,
energy balance, mirror symmetry of a car, the static axle-load split.  None
retypes the formula.  Each is chosen so that a plausible slip in the
transcription fails: swapped sin/cos, a wrong sign, a neighbour index off by
one, a dropped or swapped axle term.
"""
import math

import numpy as np
import pytest

import workloads as W

RNG = np.random.default_rng(20260)


# ------------------------------------------------------------------ unicycle

def _uni():
    return W.unicycle3d(nxy=6, ntheta=6)


def test_unicycle_heading_zero_moves_along_x_only(orc):
    p = _uni()
    tau = p.params[0]
    for v in (0.25, 1.0):
        mu = orc.mean(p, [1.2, -0.7, 0.0], [v, 0.0])
        assert mu[0] == pytest.approx(1.2 + tau * v, abs=1e-15)
        assert mu[1] == -0.7
        assert mu[2] == 0.0


def test_unicycle_heading_quarter_turn_moves_along_y_only(orc):
    p = _uni()
    tau = p.params[0]
    mu = orc.mean(p, [1.2, -0.7, math.pi / 2], [1.0, 0.0])
    assert mu[0] == pytest.approx(1.2, abs=1e-15)
    assert mu[1] == pytest.approx(-0.7 + tau, abs=1e-15)
    mu = orc.mean(p, [1.2, -0.7, -math.pi / 2], [1.0, 0.0])
    assert mu[1] == pytest.approx(-0.7 - tau, abs=1e-15)


def test_unicycle_moves_distance_tau_v_in_heading_direction(orc):
    # any heading: the planar step has length tau v and points along theta
    p = _uni()
    tau = p.params[0]
    for _ in range(50):
        x = [RNG.uniform(-4, 4), RNG.uniform(-4, 4), RNG.uniform(-3.1, 3.1)]
        v = RNG.uniform(0.05, 1.0)
        mu = orc.mean(p, x, [v, RNG.uniform(-1, 1)])
        dx, dy = mu[0] - x[0], mu[1] - x[1]
        assert math.hypot(dx, dy) == pytest.approx(tau * v, rel=1e-12)
        assert math.atan2(dy, dx) == pytest.approx(x[2], abs=1e-10)


def test_unicycle_speed_zero_stays_and_turn_rate_only_turns(orc):
    p = _uni()
    tau = p.params[0]
    for om in (-1.0, -0.3, 0.0, 0.8):
        mu = orc.mean(p, [0.4, 2.0, 1.1], [0.0, om])
        assert mu[0] == 0.4 and mu[1] == 2.0
        assert mu[2] == pytest.approx(1.1 + tau * om, abs=1e-15)
    # the turn rate never moves the position; the speed never turns
    a = orc.mean(p, [0.4, 2.0, 1.1], [0.7, -1.0])
    b = orc.mean(p, [0.4, 2.0, 1.1], [0.7, 1.0])
    assert a[0] == b[0] and a[1] == b[1]
    c = orc.mean(p, [0.4, 2.0, 1.1], [0.2, 0.5])
    d = orc.mean(p, [0.4, 2.0, 1.1], [0.9, 0.5])
    assert c[2] == d[2]


def test_unicycle_rotation_equivariance(orc):
    # rotating the plane by phi rotates the step and adds phi to the heading
    p = _uni()
    for _ in range(20):
        x = np.array([RNG.uniform(-3, 3), RNG.uniform(-3, 3), RNG.uniform(-1, 1)])
        u = [RNG.uniform(0, 1), RNG.uniform(-1, 1)]
        phi = RNG.uniform(-1.5, 1.5)
        c, s = math.cos(phi), math.sin(phi)
        xr = np.array([c * x[0] - s * x[1], s * x[0] + c * x[1], x[2] + phi])
        mu = orc.mean(p, x, u)
        mur = orc.mean(p, xr, u)
        want = [c * mu[0] - s * mu[1], s * mu[0] + c * mu[1], mu[2] + phi]
        assert np.allclose(mur, want, atol=1e-12)


# --------------------------------------------------------------- room ring

def _ring(n=5, params=None):
    p = W.room5d(cells=3, n=n)
    return p if params is None else p.with_(params=params)


# the workload's coefficients and the paper's 5-room study's (Sec. 8.2)
RING_PARAMS = [(0.05, 0.005, 0.01, -1.0, 50.0), (0.3, 0.022, 0.05, -1.0, 50.0)]


@pytest.mark.parametrize("params", RING_PARAMS)
@pytest.mark.parametrize("n", [3, 5])
def test_ring_outdoor_temperature_is_equilibrium_without_heat(orc, n, params):
    p = _ring(n, params)
    Te = params[3]
    mu = orc.mean(p, [Te] * n, [0.0])
    assert np.allclose(mu, Te, atol=1e-13)


@pytest.mark.parametrize("params", RING_PARAMS)
def test_ring_conduction_is_local_symmetric_and_circular(orc, params):
    # raising room j by d changes, with the heater off, room j and its two
    # ring neighbours only; both neighbours gain the same; rooms 0 and n-1
    # are neighbours (the rooms sit on a circle)
    n = 5
    p = _ring(n, params)
    base = np.array([20.1, 19.4, 20.7, 19.9, 20.3])
    d = 0.25
    mu0 = orc.mean(p, base, [0.0])
    for j in range(n):
        x = base.copy()
        x[j] += d
        dm = orc.mean(p, x, [0.0]) - mu0
        nb = {(j - 1) % n, (j + 1) % n}
        for i in range(n):
            if i != j and i not in nb:
                assert abs(dm[i]) < 1e-13, (j, i, dm)
        left, right = dm[(j - 1) % n], dm[(j + 1) % n]
        assert left > 0 and left == pytest.approx(right, rel=1e-9)
        assert 0 < dm[j] < d


@pytest.mark.parametrize("params", RING_PARAMS)
def test_ring_energy_balance(orc, params):
    # with the heater off, conduction between rooms moves heat but creates
    # none: the total changes only by the exchange with the outside,
    # sum mu = (1 - beta) sum x + n beta T_e
    n = 5
    p = _ring(n, params)
    al, be, ga, Te, Th = params
    for _ in range(20):
        x = RNG.uniform(19, 21, size=n)
        mu = orc.mean(p, x, [0.0])
        assert mu.sum() == pytest.approx((1 - be) * x.sum() + n * be * Te, rel=1e-14)


@pytest.mark.parametrize("params", RING_PARAMS)
def test_ring_rotation_equivariance(orc, params):
    n = 5
    p = _ring(n, params)
    for _ in range(10):
        x = RNG.uniform(19, 21, size=n)
        u = [RNG.uniform(0, 1)]
        mu = orc.mean(p, x, u)
        for r in range(1, n):
            assert np.allclose(orc.mean(p, np.roll(x, r), u), np.roll(mu, r), atol=1e-13)


@pytest.mark.parametrize("params", RING_PARAMS)
def test_ring_heater_pulls_each_room_toward_heater_temperature(orc, params):
    # the heater's effect on room i is the exchange gam u (T_h - x_i):
    # linear in u, proportional to the gap to T_h, zero at T_h
    n = 5
    p = _ring(n, params)
    al, be, ga, Te, Th = params
    x = RNG.uniform(19, 21, size=n)
    m0 = orc.mean(p, x, [0.0])
    for u in (0.25, 0.5, 1.0):
        dm = orc.mean(p, x, [u]) - m0
        assert np.all(dm > 0)
        assert np.allclose(dm / (Th - x), ga * u, rtol=1e-12)
    xh = x.copy()
    xh[2] = Th
    assert orc.mean(p, xh, [1.0])[2] == pytest.approx(orc.mean(p, xh, [0.0])[2], abs=1e-12)


def test_ring_one_heater_per_room(orc):
    # m = n heaters: heater k acts on room k alone
    n = 3
    p = _ring(n).with_(u_lo=(0.0,) * n, u_hi=(1.0,) * n, u_count=(2,) * n)
    x = np.array([19.5, 20.5, 20.0])
    m0 = orc.mean(p, x, [0.0, 0.0, 0.0])
    for k in range(n):
        u = [0.0] * n
        u[k] = 1.0
        dm = orc.mean(p, x, u) - m0
        assert dm[k] > 0 and all(abs(dm[i]) < 1e-13 for i in range(n) if i != k)


# ------------------------------------------------------------------ vehicle

def _car():
    return W.vehicle7d(cells=3)


def _rates(p, x, u):
    """(mu - x) / tau: the printed right-hand sides a_i / b_i."""
    tau = p.params[0]
    return (orc_mean(p, x, u) - np.asarray(x, float)) / tau


orc_mean = None


@pytest.fixture(autouse=True)
def _bind(orc):
    global orc_mean
    orc_mean = orc.mean


def test_vehicle_standstill(orc):
    # at zero speed the car does not move, turn or slip; steering angle and
    # speed integrate the (saturated) inputs
    p = _car()
    tau = p.params[0]
    x = [3.0, -2.0, 0.1, 0.0, 0.2, 0.0, 0.0]
    for u in ([0.2, 2.0], [-0.4, -4.0], [0.0, 0.0]):
        mu = orc.mean(p, x, u)
        assert mu[0] == 3.0 and mu[1] == -2.0 and mu[4] == 0.2 and mu[6] == 0.0
        assert mu[2] == pytest.approx(0.1 + tau * u[0], abs=1e-15)
        assert mu[3] == pytest.approx(tau * u[1], abs=1e-15)


def test_vehicle_inputs_saturate_at_input_box(orc):
    p = _car()
    x = [0.0, 0.0, 0.0, 0.05, 0.0, 0.0, 0.0]
    a = orc.mean(p, x, [5.0, 50.0])
    b = orc.mean(p, x, [p.u_hi[0], p.u_hi[1]])
    assert np.array_equal(a, b)
    a = orc.mean(p, x, [-5.0, -50.0])
    b = orc.mean(p, x, [p.u_lo[0], p.u_lo[1]])
    assert np.array_equal(a, b)


@pytest.mark.parametrize("speed", [0.06, -0.08, 1.5, -1.2])
def test_vehicle_moves_at_its_speed_along_its_course(orc, speed):
    # kinematic branch (|v| < 0.1): course = yaw angle; dynamic branch: course
    # = yaw angle + slip angle; the step length is tau |v|
    p = _car()
    tau = p.params[0]
    for _ in range(10):
        yaw, slip = RNG.uniform(-1.2, 1.2), RNG.uniform(-0.04, 0.04)
        x = [1.0, 2.0, RNG.uniform(-0.3, 0.3), speed, yaw, RNG.uniform(-0.3, 0.3), slip]
        mu = orc.mean(p, x, [0.1, 1.0])
        dx, dy = mu[0] - x[0], mu[1] - x[1]
        course = yaw + (slip if abs(speed) >= 0.1 else 0.0)
        assert math.hypot(dx, dy) == pytest.approx(tau * abs(speed), rel=1e-12)
        s = 1.0 if speed > 0 else -1.0
        assert math.atan2(s * dy, s * dx) == pytest.approx(course, abs=1e-10)


def test_vehicle_kinematic_yaw_rate_follows_bicycle_geometry(orc):
    # low speed: the yaw angle turns at v tan(delta) / l_wb, and the yaw-rate
    # state follows the time derivative of that rate as the speed and the
    # steering angle change at the inputs' rates (chain rule, checked by a
    # difference quotient of the yaw-angle rate itself)
    p = _car()
    lwb = p.params[1]
    for _ in range(20):
        d, v = RNG.uniform(-0.35, 0.35), RNG.uniform(-0.09, 0.09)
        u = [RNG.uniform(-0.4, 0.4), RNG.uniform(-4, 4)]
        x = [0.0, 0.0, d, v, 0.3, 0.1, 0.0]
        r = _rates(p, x, u)
        assert r[4] == pytest.approx(v * math.tan(d) / lwb, rel=1e-9, abs=1e-15)
        eps = 1e-6

        def yaw_rate(dd, vv):
            return _rates(p, [0.0, 0.0, dd, vv, 0.3, 0.1, 0.0], u)[4]
        num = (yaw_rate(d + eps * u[0], v + eps * u[1]) - yaw_rate(d - eps * u[0], v - eps * u[1])) / (2 * eps)
        assert r[5] == pytest.approx(num, rel=1e-5, abs=1e-9)
        assert r[6] == 0.0


def test_vehicle_dynamic_yaw_angle_integrates_yaw_rate(orc):
    p = _car()
    for _ in range(10):
        x = [0, 0, RNG.uniform(-0.3, 0.3), RNG.uniform(0.5, 2.0), RNG.uniform(-0.3, 0.3),
             RNG.uniform(-0.4, 0.4), RNG.uniform(-0.04, 0.04)]
        assert _rates(p, x, [0.0, 0.0])[4] == pytest.approx(x[5], rel=1e-9)


@pytest.mark.parametrize("speed", [0.05, 1.3])
def test_vehicle_mirror_symmetry(orc, speed):
    # reflecting the world across the x1 axis flips the lateral position, the
    # steering, yaw, yaw rate, slip and the steering input; the car has no
    # handedness, so the step is reflected the same way
    p = _car()
    flip = np.array([1, -1, -1, 1, -1, -1, -1], float)
    for _ in range(20):
        x = np.array([RNG.uniform(-5, 5), RNG.uniform(-5, 5), RNG.uniform(-0.3, 0.3), speed,
                      RNG.uniform(-0.3, 0.3), RNG.uniform(-0.4, 0.4), RNG.uniform(-0.04, 0.04)])
        u = np.array([RNG.uniform(-0.4, 0.4), RNG.uniform(-4, 4)])
        mu = orc.mean(p, x, u)
        mur = orc.mean(p, flip * x, u * np.array([-1.0, 1.0]))
        assert np.allclose(mur, flip * mu, rtol=1e-12, atol=1e-14)


def test_vehicle_straight_driving_stays_straight(orc):
    # no steering, no yaw rate, no slip: no yaw acceleration and no slip change
    p = _car()
    for v in (0.5, 1.9):
        for a in (-4.0, 0.0, 4.0):
            r = _rates(p, [0, 0, 0.0, v, 0.2, 0.0, 0.0], [0.0, a])
            assert r[5] == 0.0 and r[6] == 0.0 and r[4] == 0.0


def test_vehicle_steering_turns_and_yaw_is_damped(orc):
    # forward speed: steering left (positive angle) accelerates the yaw to the
    # left and turns the velocity to the left; a yaw rate on its own is
    # damped by the tyre forces
    p = _car()
    for v in (0.5, 1.5):
        r = _rates(p, [0, 0, 0.2, v, 0.0, 0.0, 0.0], [0.0, 0.0])
        assert r[5] > 0 and r[6] > 0
        r = _rates(p, [0, 0, 0.0, v, 0.0, 0.3, 0.0], [0.0, 0.0])
        assert r[5] < 0


def test_vehicle_static_axle_loads_make_slip_yaw_neutral(orc):
    # without acceleration the axle loads are m g l_r/(l_f+l_r) front and
    # m g l_f/(l_f+l_r) rear, so with equal cornering stiffness the two
    # axles' lateral forces from a slip angle have equal and opposite moments
    # about the centre of gravity: the slip angle alone gives no yaw
    # acceleration.  Under acceleration the load moves to the rear axle and
    # the slip angle yaws the car (swapping the axle terms breaks both).
    p = _car()
    assert p.params[8] == p.params[9]
    for v in (0.5, 1.7):
        base = _rates(p, [0, 0, 0.0, v, 0.0, 0.0, 0.0], [0.0, 0.0])[5]
        slip = _rates(p, [0, 0, 0.0, v, 0.0, 0.0, 0.03], [0.0, 0.0])[5]
        assert abs(slip - base) < 1e-12
        acc = _rates(p, [0, 0, 0.0, v, 0.0, 0.0, 0.03], [0.0, 3.0])[5]
        assert acc > 1e-6


def test_vehicle_acceleration_unloads_front_axle(orc):
    # braking (negative longitudinal acceleration) loads the front axle, so the
    # same steering angle gives a larger yaw acceleration than when accelerating
    p = _car()
    hi = _rates(p, [0, 0, 0.2, 1.0, 0.0, 0.0, 0.0], [0.0, -4.0])[5]
    mid = _rates(p, [0, 0, 0.2, 1.0, 0.0, 0.0, 0.0], [0.0, 0.0])[5]
    lo = _rates(p, [0, 0, 0.2, 1.0, 0.0, 0.0, 0.0], [0.0, 4.0])[5]
    assert hi > mid > lo > 0


def test_vehicle_branch_switch_at_speed_one_tenth(orc):
    # the model switches from the kinematic to the dynamic form at |v| = 0.1:
    # the course picks up the slip angle exactly there
    p = _car()
    for v, dyn in ((0.0999999, False), (0.1, True), (-0.1, True), (-0.0999999, False)):
        x = [0, 0, 0.0, v, 0.0, 0.0, 0.03]
        mu = orc.mean(p, x, [0.0, 0.0])
        s = 1.0 if v > 0 else -1.0
        ang = math.atan2(s * mu[1], s * mu[0])
        assert ang == pytest.approx(0.03 if dyn else 0.0, abs=1e-12)


def test_vehicle_course_kept_without_net_lateral_force(orc):
    # a car that only yaws (no steering, no slip) at static axle loads has
    # front and rear tyre slip angles -l_f r/v and +l_r r/v on axle loads in
    # the ratio l_r : l_f, so with equal cornering stiffness the two lateral
    # forces cancel; the velocity direction (yaw + slip) then does not turn,
    # so the slip angle changes at minus the yaw rate
    p = _car()
    for v in (0.6, 1.8):
        for r in (-0.3, 0.2):
            rates = _rates(p, [0, 0, 0.0, v, 0.1, r, 0.0], [0.0, 0.0])
            assert rates[4] + rates[6] == pytest.approx(0.0, abs=1e-12)
            assert rates[6] == pytest.approx(-r, rel=1e-12)
