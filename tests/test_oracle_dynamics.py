"""Pins of the RK4 rollout against closed forms (Section III feasibility,
Section V robot models)."""
import numpy as np

from oracle import dynamics
from paper_2503_12204_amd import workloads as W


def _prob(dyn, **kw):
    if dyn == W.UNICYCLE:
        base = dict(u_lo=(-1.0, -np.pi, 0.0), u_hi=(1.0, np.pi, 0.0), v_max=0.0)
    elif dyn == W.DIFFDRIVE:
        base = dict(W.DIFFDRIVE_LIMITS)
    else:
        base = dict(u_lo=(-1.0,) * 3, u_hi=(1.0,) * 3, v_max=2.0)
    base.update(kw)
    return W.Problem(dyn=dyn, **base)


def test_double_integrator_step_is_exact():
    rng = np.random.default_rng(0)
    for dyn, dp in ((W.HOLO2D, 2), (W.HOLO3D, 3)):
        p = _prob(dyn, v_max=1e9)
        x = rng.normal(size=(50, 2 * dp))
        u = rng.uniform(-1, 1, size=(50, dp))
        dt = 0.1
        xn = dynamics.step(p, x, u)
        pos = x[:, :dp] + x[:, dp:] * dt + 0.5 * u * dt * dt
        vel = x[:, dp:] + u * dt
        assert np.allclose(xn[:, :dp], pos, rtol=0, atol=1e-14)
        assert np.allclose(xn[:, dp:], vel, rtol=0, atol=1e-14)


def test_double_integrator_constant_accel_trajectory():
    p = _prob(W.HOLO2D, horizon=30)
    x0 = np.array([[1.0, -2.0, 0.5, -0.25]])
    a = np.array([0.3, -0.5])
    u = np.broadcast_to(a, (1, 1, 30, 2))
    x = dynamics.rollout(p, x0, u)
    t = np.arange(31)[:, None] * 0.1
    v = x0[0, 2:] + a * t
    assert np.abs(v).max() < 2.0  # the speed limit never binds here
    pos = x0[0, :2] + x0[0, 2:] * t + 0.5 * a * t * t
    assert np.allclose(x[0, 0, :, :2], pos, atol=1e-12)
    assert np.allclose(x[0, 0, :, 2:], v, atol=1e-12)


def test_speed_limit_and_control_clip():
    p = _prob(W.HOLO2D, horizon=40)
    x0 = np.zeros((1, 4))
    u = np.full((1, 1, 40, 2), 5.0)       # clipped to 1
    x = dynamics.rollout(p, x0, u)
    assert np.allclose(x[0, 0, 10, 2:], 1.0)        # v = a t with a = 1
    assert np.allclose(x[0, 0, 25:, 2:], 2.0)       # capped at v_max
    assert np.all(np.abs(x[..., 2:]) <= 2.0)


def test_unicycle_straight_line_exact():
    p = _prob(W.UNICYCLE, horizon=20)
    th = 0.7
    x0 = np.array([[0.5, -1.0, th]])
    u = np.zeros((1, 1, 20, 2))
    u[..., 0] = 0.8
    x = dynamics.rollout(p, x0, u)
    t = np.arange(21) * 0.1
    assert np.allclose(x[0, 0, :, 0], 0.5 + 0.8 * t * np.cos(th), atol=1e-13)
    assert np.allclose(x[0, 0, :, 1], -1.0 + 0.8 * t * np.sin(th), atol=1e-13)
    assert np.allclose(x[0, 0, :, 2], th, atol=0)


def test_unicycle_rk4_is_simpson_and_close_to_arc():
    rng = np.random.default_rng(1)
    p = _prob(W.UNICYCLE)
    dt = 0.1
    x = np.column_stack([rng.normal(size=200), rng.normal(size=200), rng.uniform(-4, 4, 200)])
    v = rng.uniform(-1, 1, 200)
    om = rng.uniform(-np.pi, np.pi, 200)
    om[:5] = [1e-3, -1e-3, 2.0, -2.0, np.pi]
    xn = dynamics.step(p, x, np.column_stack([v, om]))
    th = x[:, 2]
    # Simpson's rule on the heading, which is linear in time over the step
    simp_x = x[:, 0] + dt / 6 * v * (np.cos(th) + 4 * np.cos(th + om * dt / 2) + np.cos(th + om * dt))
    simp_y = x[:, 1] + dt / 6 * v * (np.sin(th) + 4 * np.sin(th + om * dt / 2) + np.sin(th + om * dt))
    assert np.allclose(xn[:, 0], simp_x, atol=1e-14)
    assert np.allclose(xn[:, 1], simp_y, atol=1e-14)
    assert np.allclose(xn[:, 2], th + om * dt, atol=1e-14)
    # exact circular arc and Simpson's error bound |v| omega^4 dt^5 / 2880
    arc_x = x[:, 0] + v / om * (np.sin(th + om * dt) - np.sin(th))
    arc_y = x[:, 1] - v / om * (np.cos(th + om * dt) - np.cos(th))
    # plus rounding of the arc formula, amplified by v / omega for slow turns
    bound = np.abs(v) * om ** 4 * dt ** 5 / 2880 + 1e-15 * (1 + np.abs(v / om))
    assert np.all(np.abs(xn[:, 0] - arc_x) <= bound)
    assert np.all(np.abs(xn[:, 1] - arc_y) <= bound)


def test_zero_control_rest_and_translation():
    rng = np.random.default_rng(2)
    for dyn in (W.HOLO2D, W.HOLO3D, W.UNICYCLE, W.DIFFDRIVE):
        p = _prob(dyn, horizon=15)
        dx, du, dp = W.dims(dyn)
        x0 = np.zeros((3, dx))
        x0[:, :dp] = rng.normal(size=(3, dp))
        if dyn in (W.UNICYCLE, W.DIFFDRIVE):
            x0[:, 2] = rng.uniform(-3, 3, 3)
        x = dynamics.rollout(p, x0, np.zeros((1, 3, 15, du)))
        assert np.array_equal(x[0], np.broadcast_to(x0[:, None, :], (3, 16, dx)))
        u = rng.uniform(-1.5, 1.5, size=(2, 3, 15, du))
        shift = np.zeros(dx)
        shift[:dp] = rng.normal(size=dp) * 5
        xa = dynamics.rollout(p, x0, u)
        xb = dynamics.rollout(p, x0 + shift, u)
        assert np.allclose(xb - shift, xa, atol=1e-12)


def test_diffdrive_straight_line_constant_acceleration_exact():
    """omega = 0: the heading stays, the speed grows linearly and the position
    follows v0 t + a t^2 / 2 along the heading; RK4 (Simpson on a linear
    integrand) is exact while the speed bound does not bind."""
    p = _prob(W.DIFFDRIVE, horizon=20)
    th, v0, a = -1.1, 0.2, 0.35
    x0 = np.array([[0.5, -1.0, th, v0]])
    u = np.zeros((1, 1, 20, 2))
    u[..., 1] = a
    x = dynamics.rollout(p, x0, u)
    t = np.arange(21) * 0.1
    assert np.abs(v0 + a * t).max() < 1.0
    s = v0 * t + 0.5 * a * t * t
    assert np.allclose(x[0, 0, :, 0], 0.5 + s * np.cos(th), atol=1e-13)
    assert np.allclose(x[0, 0, :, 1], -1.0 + s * np.sin(th), atol=1e-13)
    assert np.allclose(x[0, 0, :, 2], th, atol=0)
    assert np.allclose(x[0, 0, :, 3], v0 + a * t, atol=1e-14)


def test_diffdrive_rk4_is_simpson_and_close_to_arc():
    """Constant turn rate and acceleration over a step: theta and v are linear
    in time, the RK4 stages k2 = k3, and the position update is Simpson's rule
    on v(s) cos theta(s); at a = 0 it stays within Simpson's bound of the arc."""
    rng = np.random.default_rng(4)
    p = _prob(W.DIFFDRIVE, v_max=1e9)
    dt = 0.1
    n = 200
    x = np.column_stack([rng.normal(size=n), rng.normal(size=n), rng.uniform(-4, 4, n), rng.uniform(-1, 1, n)])
    om = rng.uniform(-np.pi, np.pi, n)
    om[:5] = [1e-3, -1e-3, 2.0, -2.0, np.pi]
    a = rng.uniform(-1, 1, n)
    xn = dynamics.step(p, x, np.column_stack([om, a]))
    th, v = x[:, 2], x[:, 3]
    vh, v1 = v + a * dt / 2, v + a * dt
    simp_x = x[:, 0] + dt / 6 * (v * np.cos(th) + 4 * vh * np.cos(th + om * dt / 2) + v1 * np.cos(th + om * dt))
    simp_y = x[:, 1] + dt / 6 * (v * np.sin(th) + 4 * vh * np.sin(th + om * dt / 2) + v1 * np.sin(th + om * dt))
    assert np.allclose(xn[:, 0], simp_x, atol=1e-14)
    assert np.allclose(xn[:, 1], simp_y, atol=1e-14)
    assert np.allclose(xn[:, 2], th + om * dt, atol=1e-14)
    assert np.allclose(xn[:, 3], v1, atol=1e-15)
    # a = 0: a circular arc of radius v / omega, within Simpson's error bound
    x0 = x.copy()
    xn = dynamics.step(p, x0, np.column_stack([om, np.zeros(n)]))
    arc_x = x0[:, 0] + v / om * (np.sin(th + om * dt) - np.sin(th))
    arc_y = x0[:, 1] - v / om * (np.cos(th + om * dt) - np.cos(th))
    bound = np.abs(v) * om ** 4 * dt ** 5 / 2880 + 1e-15 * (1 + np.abs(v / om))
    assert np.all(np.abs(xn[:, 0] - arc_x) <= bound)
    assert np.all(np.abs(xn[:, 1] - arc_y) <= bound)


def test_diffdrive_speed_bound():
    """The speed is clipped to [-v_max, v_max] after each step; the turn-rate
    and acceleration controls are clipped to their box first."""
    p = _prob(W.DIFFDRIVE, horizon=40)
    x0 = np.zeros((1, 4))
    u = np.zeros((1, 1, 40, 2))
    u[..., 1] = 5.0                                   # clipped to a = 1
    x = dynamics.rollout(p, x0, u)
    assert np.allclose(x[0, 0, 5, 3], 0.5)            # v = a t
    assert np.allclose(x[0, 0, 10:, 3], 1.0)          # capped at v_max = 1
    assert np.all(np.abs(x[..., 3]) <= 1.0)
    # once capped, every step starts at v_max and integrates v(s) = v_max + a s
    # (the bound applies after the step): dt v_max + a dt^2 / 2 = 0.105 m
    assert np.allclose(np.diff(x[0, 0, 12:, 0]), 0.105, atol=1e-14)
