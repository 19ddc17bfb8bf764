"""Pins of the Monte Carlo score update (Eqs. denoising, guidance, mc,
mbd-denoising; Algorithms 1 and 2)."""
import numpy as np

from oracle import dynamics, mbd, noise, schedule
from paper_2503_12204_amd import workloads as W


def test_weights_sum_to_one_and_degenerate_cases():
    rng = np.random.default_rng(0)
    r = rng.normal(size=1000)
    for norm in (True, False):
        w = mbd.weights(r, 0.1, norm)
        assert abs(w.sum() - 1) < 1e-12 and (w >= 0).all()
    w = mbd.weights(np.full(37, 0.3), 0.1, True)
    assert np.allclose(w, 1 / 37, atol=1e-15)
    w = mbd.weights(r, 1e12, True)
    assert np.allclose(w, 1 / 1000, rtol=1e-9)
    # argmax limit as the temperature vanishes (distinct rewards)
    w = mbd.weights(r, 1e-6, False)
    assert w[np.argmax(r)] > 1 - 1e-12


def test_normalised_weights_equal_plain_weights_at_scaled_temperature():
    rng = np.random.default_rng(1)
    r = rng.normal(size=500) * 0.03 + 0.4
    sd = np.sqrt(((r - r.mean()) ** 2).mean())
    assert np.allclose(mbd.weights(r, 0.1, True), mbd.weights(r, 0.1 * sd, False), rtol=1e-10)


def _is_stats(samples, w):
    ubar = (w[:, None] * samples).sum(0)
    se = np.sqrt((w[:, None] ** 2 * (samples - ubar) ** 2).sum(0))
    return ubar, se


def test_linear_fitness_exponential_tilt():
    """r = g.u: the weighted mean of N(mu, s2 I) samples tends to mu + s2 g / lambda."""
    rng = np.random.default_rng(2)
    D, M, lam = 4, 400_000, 0.5
    mu = rng.normal(size=D)
    g = rng.normal(size=D) * 0.3
    ms_i, sg_i = 1.3, 0.7
    du_i = mu / ms_i
    eps = rng.normal(size=(D, M))
    samples = mbd.sample_deformations(du_i, eps, ms_i, sg_i)
    r = samples @ g
    du_next, w = mbd.mc_update(du_i, eps, r, ms_i, sg_i, 1.0, lam, normalize=False)
    expect = mu + sg_i ** 2 * g / lam
    _, se = _is_stats(samples, w)
    assert np.all(np.abs(du_next - expect) <= 4 * se + 1e-12)


def test_linear_fitness_through_all_denoising_steps():
    """Algorithm 1 over all N steps with r = c.u: each step's weighted mean is the
    exponential tilt (Eq. mc with Gaussian draws), so V_i = Delta U_i / sqrt(abar_i)
    gains sigma_i^2 c / lambda per step and Delta U_0 = sum_i sigma_i^2 c / lambda
    (abar_0 = 1).  This pins the chained update and the schedule's scales
    against each other: an out scale sqrt(abar_i) in place of sqrt(abar_{i-1}),
    or a mean scale of the wrong step, misses it by about nine times the
    Monte Carlo tolerance, a sigma of the wrong step by about twice."""
    rng = np.random.default_rng(6)
    N, D, M, lam = 100, 4, 20_000, 0.1
    ms, sg, os_ = schedule.step_scalars(N, 1e-4, 1e-2)
    ab = schedule.alpha_bar(N, 1e-4, 1e-2)
    c = np.array([0.08, -0.04, 0.0, 0.02])
    du = np.zeros(D)
    for i in range(N, 0, -1):
        eps = rng.normal(size=(D, M))
        samples = mbd.sample_deformations(du, eps, ms[i], sg[i])
        du, _ = mbd.mc_update(du, eps, samples @ c, ms[i], sg[i], os_[i], lam, normalize=False)
    s2 = sum(1.0 / ab[i] - 1.0 for i in range(1, N + 1))
    expect = s2 * c / lam
    # each step adds sigma_i times a self-normalised weighted mean of M standard
    # normals; exponential weights of tilt a inflate its variance by exp(|a|^2)
    a_max = np.sqrt(1.0 / ab[N] - 1.0) * np.linalg.norm(c) / lam
    tol = 6.0 * np.sqrt(s2 * np.exp(a_max ** 2) / M)
    assert np.all(np.abs(du - expect) <= tol), (du, expect, tol)
    assert abs(expect[0]) > 50 * tol


def test_planner_loop_with_a_linear_fitness(monkeypatch):
    """The oracle's own Algorithm 2 loop body (denoise_iteration: Delta U_N = 0,
    steps N..1 with its Philox draws, then the apply step) with the robot
    fitness swapped for r = c.u on unclipped controls: Delta U_0 must be the
    closed form sum_i sigma_i^2 c / lambda of the linear-fitness pin above.
    Steps taken in increasing order miss it by about three times the
    tolerance, an index off by one by far more."""
    from oracle import fitness
    p, x0, g = W.holo2d_circle(n=1, horizon=2, n_samples=20_000)
    p = p.replace(flags=0, temperature=0.1)
    M, D = p.n_samples, p.D
    c = np.array([0.08, -0.04, 0.0, 0.02])
    monkeypatch.setattr(dynamics, "clip_controls", lambda prob, u: u)
    monkeypatch.setattr(dynamics, "rollout", lambda prob, x0_, u: np.asarray(u, dtype=np.float64))
    monkeypatch.setattr(fitness, "reward", lambda prob, x, goal, pred_dtype=np.float64: (
        x.reshape(x.shape[0], -1) @ c, np.zeros(x.shape[0], int), np.zeros(x.shape[0], int)))
    for name in ("success", "at_goal", "objective"):
        monkeypatch.setattr(fitness, name, lambda prob, x, goal: np.zeros(x.shape[0]))
    res = mbd.denoise_iteration(p, x0, g, np.zeros(D), 0)
    ab = schedule.alpha_bar(p.n_steps, p.beta_min, p.beta_max)
    s2 = sum(1.0 / ab[i] - 1.0 for i in range(1, p.n_steps + 1))
    expect = s2 * c / p.temperature
    a_max = np.sqrt(1.0 / ab[p.n_steps] - 1.0) * np.linalg.norm(c) / p.temperature
    tol = 6.0 * np.sqrt(s2 * np.exp(a_max ** 2) / M)
    assert np.all(np.abs(res["du0"] - expect) <= tol), (res["du0"], expect, tol)
    assert np.allclose(res["u"].reshape(-1), res["du0"])


def test_quadratic_fitness_posterior_and_smoothed_score():
    """r = -|u - u*|^2 / (2 s): the MC mean tends to the Gaussian posterior mean,
    and Eq. guidance with that mean is the exact score of the noised density."""
    rng = np.random.default_rng(3)
    D, M, lam, s = 5, 400_000, 0.5, 4.0
    sched = schedule.step_scalars(100, 1e-4, 1e-2)
    ab = schedule.alpha_bar(100, 1e-4, 1e-2)
    i = 60
    ms, sg, os_ = sched[0][i], sched[1][i], sched[2][i]
    tau_i = rng.normal(size=D)
    ustar = rng.normal(size=D)
    eps = rng.normal(size=(D, M))
    samples = mbd.sample_deformations(tau_i, eps, ms, sg)
    r = -((samples - ustar) ** 2).sum(1) / (2 * s)
    tau_prev, w = mbd.mc_update(tau_i, eps, r, ms, sg, os_, lam, normalize=False)
    mu, s2 = tau_i * ms, sg ** 2
    post = (s * lam * mu + s2 * ustar) / (s * lam + s2)
    _, se = _is_stats(samples, w)
    assert np.all(np.abs(tau_prev / os_ - post) <= 4 * se)
    # Eq. guidance with the posterior mean equals the score of p_i = p_0 * forward noise
    a = ab[i]
    guided = -tau_i / (1 - a) + np.sqrt(a) / (1 - a) * post
    exact = (np.sqrt(a) * ustar - tau_i) / (a * s * lam + 1 - a)
    assert np.allclose(guided, exact, rtol=1e-12, atol=1e-12)
    # Eq. denoising with that score equals Eq. mbd-denoising
    alpha_i = a / ab[i - 1]
    denoised = (tau_i + (1 - a) * guided) / np.sqrt(alpha_i)
    assert np.allclose(denoised, np.sqrt(ab[i - 1]) * post, rtol=1e-12)


def test_zero_spread_is_pure_rescale():
    du_i = np.array([0.3, -1.2, 2.0])
    out, _ = mbd.mc_update(du_i, np.ones((3, 8)), np.arange(8.0), 1.7, 0.0, 0.9, 0.1)
    assert np.allclose(out, 0.9 * 1.7 * du_i, rtol=1e-15)


def test_dimension_count_and_rollout_count(monkeypatch):
    # 16 2D-holonomic robots at H = 100 have 3200 optimisation variables
    assert W.Problem(dyn=W.HOLO2D, n_robots=16, horizon=100).D == 3200
    # K iterations of N steps roll out K*N*M sample trajectories plus K final ones
    calls = []
    orig = dynamics.rollout

    def counting(prob, x0, u):
        calls.append(np.asarray(u).shape[0])
        return orig(prob, x0, u)

    monkeypatch.setattr(dynamics, "rollout", counting)
    p, x0, g = W.holo2d_circle(n=3, horizon=6, n_samples=5)
    p = p.replace(n_steps=3)
    mbd.plan(p, x0, g, iterations=2)
    assert sum(calls) == 2 * 3 * 5 + 2


def test_step_uses_the_specified_draws():
    p, x0, g = W.holo2d_circle(n=3, horizon=5, n_samples=8)
    p = p.replace(n_steps=4, seed=77)
    D = p.D
    out = mbd.denoise_step(p, x0, g, np.zeros(D), np.zeros(D), kappa=1, i=3)
    assert np.array_equal(out["eps"], noise.draw(77, 0, 1, 3, 8, D))


def test_planner_improves_circle_swap():
    """Distribution-level sanity only (parity unpinned): one iteration on the
    4-robot circle swap must beat the zero-control start and reach the goals."""
    p, x0, g = W.holo2d_circle()
    p = p.replace(n_samples=128)
    u0 = np.zeros((p.n_robots, p.horizon, p.du))
    base = mbd.apply_deformation(p, x0, g, u0, np.zeros(p.D))
    u, hist = mbd.plan(p, x0, g, iterations=1)
    assert hist[0]["r"] > base["r"] + 0.2


def _deformation_case():
    """One 2D double integrator, two steps, a non-zero plan tau.u and a
    deformation whose sum with it leaves the control box |a| <= 1 on three of
    four components.  Expected controls and states are worked out by hand:
    clip(tau.u + Delta U) = [[1.0, -0.6], [-0.3, -1.0]], and the double
    integrator from rest gives p1 = a0 dt^2 / 2, v1 = a0 dt,
    p2 = p1 + v1 dt + a1 dt^2 / 2, v2 = v1 + a1 dt (RK4 is exact for it)."""
    p = W.Problem(dyn=W.HOLO2D, n_robots=1, horizon=2, n_samples=1, dt=0.1, v_max=2.0,
                  u_lo=(-1.0, -1.0, -1.0), u_hi=(1.0, 1.0, 1.0), flags=0)
    x0 = np.zeros((1, 4))
    goal = np.array([[1.0, 0.0]])
    tau_u = np.array([[0.7, -0.5], [0.2, -0.9]])
    du = np.array([[0.6, -0.1], [-0.5, -0.4]])
    u_expect = np.array([[1.0, -0.6], [-0.3, -1.0]])
    x_expect = np.array([[0.0, 0.0, 0.0, 0.0],
                         [0.005, -0.003, 0.1, -0.06],
                         [0.0135, -0.014, 0.07, -0.16]])
    return p, x0, goal, tau_u, du, u_expect, x_expect


def test_effective_controls_clip_the_sum_with_the_plan():
    """Algorithm 2 rolls out tau.u + Delta U^(m), clipped per component
    (reading R8): the clip applies to the sum, not to the deformation alone,
    and the plan is not dropped.  Clipping Delta U before adding tau.u gives
    [[1.3, -0.6], [-0.3, -1.3]]; dropping tau.u gives Delta U itself."""
    p, x0, goal, tau_u, du, u_expect, x_expect = _deformation_case()
    u = mbd.effective_controls(p, tau_u.reshape(-1), du.reshape(1, -1))
    assert u.shape == (1, 1, 2, 2)
    assert np.allclose(u[0, 0], u_expect, rtol=0, atol=1e-15)
    x = dynamics.rollout(p, x0, u)
    assert np.allclose(x[0, 0], x_expect, rtol=0, atol=1e-15)


def test_apply_deformation_closed_form_with_a_binding_box():
    """The iteration's update tau.u <- clip(tau.u + Delta U_0) and the rollout
    of the new plan (Algorithm 2), against the hand-worked controls and the
    double integrator's closed-form states; the reward follows Eq.
    generic-reward with d0 = |p_0 - g| = 1 and no partners."""
    p, x0, goal, tau_u, du, u_expect, x_expect = _deformation_case()
    res = mbd.apply_deformation(p, x0, goal, tau_u.reshape(-1), du.reshape(-1))
    assert np.allclose(res["u"][0], u_expect, rtol=0, atol=1e-15)
    assert np.allclose(res["x"][0], x_expect, rtol=0, atol=1e-15)
    d1 = np.hypot(1.0 - 0.005, 0.003)
    d2 = np.hypot(1.0 - 0.0135, 0.014)
    assert abs(res["r"] - ((1.0 - d1) + (1.0 - d2)) / 2.0) < 1e-15
    assert res["hits"] == 0 and res["success"] and not res["at_goal"]


def test_one_sample_step_moves_the_plan_by_its_own_deformation():
    """With M = 1 the softmax weight is 1 whatever the reward, so one
    denoising step returns sqrt(abar_{i-1}) (Delta U_i / sqrt(abar_i)
    + sigma_i eps) (Eq. mbd-denoising) and rolls out clip(tau.u + that sample)
    (Algorithm 1 sampling and rollout steps): the rollout of the step is the
    closed-form trajectory of the clipped sum."""
    p, x0, goal, tau_u, du, u_expect, x_expect = _deformation_case()
    p = p.replace(n_steps=4)
    ms, sg, os_ = schedule.step_scalars(p.n_steps, p.beta_min, p.beta_max)
    i = 3
    eps = np.array([[0.5], [-1.0], [2.0], [0.25]])
    # choose Delta U_i so that the sample equals du exactly
    du_i = (du.reshape(-1) - sg[i] * eps[:, 0]) / ms[i]
    out = mbd.denoise_step(p, x0, goal, tau_u.reshape(-1), du_i, 0, i, eps=eps)
    assert np.allclose(out["w"], [1.0])
    assert np.allclose(out["du_next"], os_[i] * du.reshape(-1), rtol=1e-14, atol=1e-15)
    assert np.allclose(out["x"][0, 0], x_expect, rtol=0, atol=1e-14)


def _swap_pair_case(n_steps):
    """Two 2D double integrators 3 m apart on the x axis, each with its goal
    4 m away past the other robot; T = 2, dt = 1, w_safe = 1, reward distance
    2 R_a + epsilon = 2.5 m, lambda = 0.5, batch-normalised rewards.  A sample
    drives both robots either toward their goals at full thrust at t = 0
    ("toward") or away from them ("away") and coasts at t = 1; its draws are
    so large that the clip decides the controls whatever sigma_i is.  Worked
    out by hand (RK4 is exact for the double integrator: p1 = p0 + a/2,
    v1 = a, p2 = p1 + v1):
      toward: robot 0 at (0.5, 0), (1.5, 0); robot 1 at (2.5, 0), (1.5, 0);
              r_goal = 1 - 3.5/4 and 1 - 2.5/4 for each robot; the robots are
              2 m and 0 m apart, r_safe = -1 for both at both steps, so
              r = (2 (0.125 + 0.375) - 4) / 4 = -0.75 and hits = 2;
      away:   robot 0 at (-0.5, 0), (-1.5, 0); robot 1 at (3.5, 0), (4.5, 0);
              r_goal = 1 - 4.5/4 and 1 - 5.5/4, no pair within 2.5 m, so
              r = 2 (-0.125 - 0.375) / 4 = -0.25 and hits = 0.
    The batch z-scores of (-0.75, -0.25) are (-1, +1), so the weights are
    exp(-4) / (1 + exp(-4)) for "toward" and 1 / (1 + exp(-4)) for "away".
    Deformation elements run e = k T d_u + t d_u + d (robot, step, axis): the
    "toward" direction is +1 on element 0 (robot 0, t = 0, a_x) and -1 on
    element 4 (robot 1, t = 0, a_x)."""
    p = W.Problem(dyn=W.HOLO2D, n_robots=2, horizon=2, n_samples=2, n_steps=n_steps, dt=1.0,
                  robot_radius=1.0, safety_margin=0.5, w_safe=1.0, temperature=0.5, v_max=2.0)
    x0 = np.array([[0.0, 0.0, 0.0, 0.0], [3.0, 0.0, 0.0, 0.0]])
    goal = np.array([[4.0, 0.0], [-1.0, 0.0]])
    toward = np.zeros(8)
    toward[0], toward[4] = 1.0, -1.0
    w_away = 1.0 / (1.0 + np.exp(-4.0))
    w_toward = np.exp(-4.0) / (1.0 + np.exp(-4.0))
    pos = {"toward": [[(0.5, 0.0), (1.5, 0.0)], [(2.5, 0.0), (1.5, 0.0)]],
           "away": [[(-0.5, 0.0), (-1.5, 0.0)], [(3.5, 0.0), (4.5, 0.0)]]}
    return p, x0, goal, toward, w_toward, w_away, pos


def test_two_sample_step_with_the_robot_fitness():
    """One denoising step of Algorithm 1 with the robot fitness of Eq.
    generic-reward on two samples: the rollouts, rewards, pair counts,
    weights and the update Delta U_{i-1} = sqrt(abar_{i-1}) sum_m w_m sigma_i
    eps^(m) (Delta U_i = 0) against the hand-worked case above.  A dropped
    safety term ranks "toward" first; deformation elements in another order,
    or a sample's rollout scored as another's, move the robots elsewhere."""
    p, x0, goal, toward, w_toward, w_away, pos = _swap_pair_case(3)
    ms, sg, os_ = schedule.step_scalars(p.n_steps, p.beta_min, p.beta_max)
    i, L = 2, 1e3
    eps = np.stack([L * toward, -L * toward], axis=1)        # [D][M]: sample 0 toward, 1 away
    out = mbd.denoise_step(p, x0, goal, np.zeros(p.D), np.zeros(p.D), 0, i, eps=eps)
    for m, key in enumerate(("toward", "away")):
        for k in range(2):
            for t in range(2):
                assert np.allclose(out["x"][m, k, t + 1, :2], pos[key][k][t], rtol=0, atol=1e-15)
    assert np.allclose(out["r"], [-0.75, -0.25], rtol=0, atol=1e-15)
    assert list(out["hits"]) == [2, 0] and list(out["robots_hit"]) == [4, 0]
    assert np.allclose(out["w"], [w_toward, w_away], rtol=1e-14, atol=0)
    expect = os_[i] * sg[i] * L * (w_toward - w_away) * toward
    assert np.allclose(out["du_next"], expect, rtol=1e-13, atol=1e-12)


def test_planner_iteration_with_the_robot_fitness(monkeypatch):
    """The oracle's Algorithm 2 loop body (denoise_iteration) and plan with the
    robot fitness, N = 2, on the hand-worked case above with the draws of each
    step fixed: step 2 offers (toward, away) and keeps mostly "away", step 1
    offers (away, toward) with draws a thousand times larger, so that its
    clip again ignores the carried deformation.  By hand:
      Delta U_1 = sqrt(abar_1) sigma_2 L (w_t - w_a) v,
      Delta U_0 = sqrt(abar_0) (Delta U_1 / sqrt(abar_1) + sigma_1 L' (w_t - w_a) v)
    (the weights sum to one, so the carried part passes through whole), with
    v the "toward" direction and w_t < w_a; the plan clip(Delta U_0) is the
    full-thrust "away" control, whose rollout scores -0.25 with no pair
    within the reward distance.  Steps visited out of order, or one step's
    update not carried into the next, miss Delta U_0."""
    p, x0, goal, toward, w_toward, w_away, _ = _swap_pair_case(2)
    ms, sg, os_ = schedule.step_scalars(p.n_steps, p.beta_min, p.beta_max)
    L, L1 = 1e3, 1e6
    draws = {2: np.stack([L * toward, -L * toward], axis=1), 1: np.stack([-L1 * toward, L1 * toward], axis=1)}
    visited = []

    def fixed_draw(seed, inst, kappa, step, M, D, samples=None):
        assert (M, D, samples) == (2, 8, None)
        visited.append(step)
        return draws[step]

    monkeypatch.setattr(noise, "draw", fixed_draw)
    res = mbd.denoise_iteration(p, x0, goal, np.zeros(p.D), 0)
    assert visited == [2, 1]
    du1 = os_[2] * sg[2] * L * (w_toward - w_away) * toward
    du0 = os_[1] * (ms[1] * du1 + sg[1] * L1 * (w_toward - w_away) * toward)
    assert np.allclose(res["du0"], du0, rtol=1e-13, atol=1e-9)
    away_u = np.zeros((2, 2, 2))
    away_u[0, 0, 0], away_u[1, 0, 0] = -1.0, 1.0
    assert np.array_equal(res["u"], away_u)
    assert abs(res["r"] + 0.25) < 1e-15 and res["hits"] == 0 and res["success"] and not res["at_goal"]
    visited.clear()
    u, hist = mbd.plan(p, x0, goal, iterations=1)
    assert visited == [2, 1] and np.array_equal(u, away_u) and abs(hist[0]["r"] + 0.25) < 1e-15
