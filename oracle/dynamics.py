"""Robot dynamics and the RK4 rollout, in FP64.

The feasibility condition of Section III steps the state with a classical
fourth-order Runge-Kutta step of x' = f_dyn(x, u) over dt, with the control
held for the step; Section IV-C rolls a control sequence out from the start
state this way.  Models (Section V and the workload definitions):

* HOLO2D: x = [p_x, p_y, v_x, v_y], u = [a_x, a_y], f = [v, a]  (double integrator)
* HOLO3D: the same in three dimensions
* UNICYCLE: x = [p_x, p_y, theta], u = [v, omega], f = [v cos theta, v sin theta, omega]
* DIFFDRIVE (the paper's differential drive, Section V): x = [p_x, p_y, theta, v],
  u = [omega, a], f = [v cos theta, v sin theta, omega, a]

Readings (the paper is silent on limits): every control component is clipped to
[u_lo, u_hi] before it is applied; holonomic velocities are clipped per
component, and the differential drive's speed v, to [-v_max, v_max] after each
full RK4 step; theta is not wrapped.

The RK4 step below is the literal four-stage formula; nothing is simplified.
Pinned by closed forms: RK4 is exact for the double integrator, reduces to
Simpson's rule for the unicycle, zero control keeps a resting team at rest,
and translation equivariance; the differential drive reduces to Simpson's rule
as well and is exact on straight lines at constant acceleration
(tests/test_oracle_dynamics.py).
"""
import numpy as np

HOLO2D, HOLO3D, UNICYCLE, DIFFDRIVE = 0, 1, 2, 3


def dims(dyn):
    """(d_x, d_u, d_p) of a dynamics id."""
    return {HOLO2D: (4, 2, 2), HOLO3D: (6, 3, 3), UNICYCLE: (3, 2, 2), DIFFDRIVE: (4, 2, 2)}[dyn]


def f_dyn(dyn, x, u):
    """Time derivative of the state; x [..., d_x], u [..., d_u]."""
    if dyn in (HOLO2D, HOLO3D):
        dp = dims(dyn)[2]
        return np.concatenate([x[..., dp:2 * dp], u], axis=-1)
    if dyn == UNICYCLE:
        v, om, th = u[..., 0], u[..., 1], x[..., 2]
        return np.stack([v * np.cos(th), v * np.sin(th), om], axis=-1)
    if dyn == DIFFDRIVE:
        om, a, th, v = u[..., 0], u[..., 1], x[..., 2], x[..., 3]
        return np.stack([v * np.cos(th), v * np.sin(th), om, a], axis=-1)
    raise ValueError(dyn)


def rk4(dyn, x, u, dt):
    """One classical Runge-Kutta step with the control held constant."""
    k1 = f_dyn(dyn, x, u)
    k2 = f_dyn(dyn, x + 0.5 * dt * k1, u)
    k3 = f_dyn(dyn, x + 0.5 * dt * k2, u)
    k4 = f_dyn(dyn, x + dt * k3, u)
    return x + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def clip_controls(prob, u):
    """Clip every control component to its box [u_lo, u_hi]."""
    du = dims(prob.dyn)[1]
    lo = np.asarray(prob.u_lo, dtype=np.float64)[:du]
    hi = np.asarray(prob.u_hi, dtype=np.float64)[:du]
    return np.minimum(np.maximum(u, lo), hi)


def step(prob, x, u):
    """x[t+1] from x[t] and an already clipped control u[t]."""
    xn = rk4(prob.dyn, x, u, float(prob.dt))
    if prob.dyn in (HOLO2D, HOLO3D):
        dp = dims(prob.dyn)[2]
        vm = float(prob.v_max)
        xn[..., dp:2 * dp] = np.minimum(np.maximum(xn[..., dp:2 * dp], -vm), vm)
    elif prob.dyn == DIFFDRIVE:
        vm = float(prob.v_max)
        xn[..., 3] = np.minimum(np.maximum(xn[..., 3], -vm), vm)
    return xn


def rollout(prob, x0, u):
    """State trajectories from starts x0 [n][d_x] and controls u [M][n][T][d_u].

    The controls are clipped first.  Returns x [M][n][T+1][d_x] in FP64 with
    x[:, :, 0] = x0.
    """
    u = clip_controls(prob, np.asarray(u, dtype=np.float64))
    M, n, T, _ = u.shape
    x0 = np.asarray(x0, dtype=np.float64)
    dx = x0.shape[-1]
    x = np.empty((M, n, T + 1, dx))
    x[:, :, 0] = np.broadcast_to(x0, (M, n, dx))
    for t in range(T):
        x[:, :, t + 1] = step(prob, x[:, :, t], u[:, :, t])
    return x
