"""Monte Carlo score denoising (Algorithm 1) on deformations (Algorithm 2).

One denoising step i (Algorithm 1, in the deformation form of Section IV-D):
  1. draw epsilon^(m) and form Delta U^(m) = Delta U_i / sqrt(alpha-bar_i)
     + sqrt(1/alpha-bar_i - 1) epsilon^(m)                     (Eq. mc, sample step)
  2. roll out clip(tau.u + Delta U^(m)) from the start states  (rollout step)
  3. rewards r^(m) of the rolled-out trajectories              (Eq. generic-reward)
  4. normalise the rewards within the batch and take weights
     w_m proportional to exp(r^(m) / lambda)                   (p_0 of Section IV-B)
  5. U-bar = sum_m w_m Delta U^(m), Delta U_{i-1} = sqrt(alpha-bar_{i-1}) U-bar
                                                               (Eq. mbd-denoising)
One iteration of Algorithm 2 starts from Delta U_N = 0 (Section IV-D), runs
steps i = N..1 and applies tau.u <- clip(tau.u + Delta U_0) followed by a rollout.

Readings: the batch normalisation is a z-score with the population standard
deviation floored at 1e-6 (flag NORMALIZE); tau is initialised with zero
controls; the M draws are i.i.d. (no extra mean sample).

Pinned by: the closed-form Gaussian tilt of a linear fitness and the
Gaussian posterior of a quadratic fitness (both reduce the MC estimate to the
smoothed score of Eq. guidance), the algebraic identity that Eqs. denoising and
guidance give Eq. mbd-denoising, weights summing to one, uniform weights for
equal rewards, the temperature identity of the normalisation, and, over all
N steps, the closed form of a linear fitness (the tilt accumulated through the
schedule) for the chained update and for the loop of denoise_iteration
(tests/test_oracle_mbd.py).  With the robot fitness, one step on two samples
and the whole loop body (two steps, then the apply step, and plan) are
pinned by a hand-worked two-robot case whose draws are large enough that the
control clip fixes every rollout: positions, rewards, pair counts, weights,
the carried deformation and the final plan are worked out by hand.  Beyond
such cases the planner's trajectories are the composition of these pinned
steps.
"""
import numpy as np

from . import dynamics, fitness, noise, schedule
from .fitness import FLAG_NORMALIZE


def normalise(r, normalize=True):
    """Batch normalisation of rewards: (r - mean) / max(std, 1e-6)."""
    r = np.asarray(r, dtype=np.float64)
    if not normalize:
        return r
    mu = r.mean()
    sd = np.sqrt(((r - mu) ** 2).mean())
    return (r - mu) / max(sd, 1e-6)


def weights(r, temperature, normalize=True):
    """w_m = exp(r_hat_m / lambda) / sum_j exp(r_hat_j / lambda)."""
    z = normalise(r, normalize) / float(temperature)
    z = z - z.max()
    e = np.exp(z)
    return e / e.sum()


def sample_deformations(du_i, eps, ms_i, sigma_i):
    """Delta U^(m) = Delta U_i * mean_scale_i + sigma_i * epsilon^(m); eps [D][M] -> [M][D]."""
    du_i = np.asarray(du_i, dtype=np.float64).reshape(-1)
    return du_i[None, :] * ms_i + sigma_i * np.asarray(eps, dtype=np.float64).T


def mc_update(du_i, eps, r, ms_i, sigma_i, os_i, temperature, normalize=True):
    """(Delta U_{i-1} [D], w [M]): the weighted mean of the samples, rescaled."""
    samples = sample_deformations(du_i, eps, ms_i, sigma_i)
    w = weights(r, temperature, normalize)
    ubar = (w[:, None] * samples).sum(axis=0)
    return os_i * ubar, w


def effective_controls(prob, u_base, samples):
    """clip(tau.u + Delta U^(m)) as [M][n][T][d_u]; samples [M][D]."""
    n, T, du = prob.n_robots, prob.horizon, dynamics.dims(prob.dyn)[1]
    u = np.asarray(u_base, dtype=np.float64).reshape(1, n, T, du) + samples.reshape(-1, n, T, du)
    return dynamics.clip_controls(prob, u)


def sample_rewards(prob, x0, goal, u_base, du_i, kappa, i, sched=None, samples=None):
    """Sampling, rollout and reward of step i for all samples or the listed ones."""
    if sched is None:
        sched = schedule.step_scalars(prob.n_steps, prob.beta_min, prob.beta_max)
    ms, sg, _ = sched
    D = prob.n_robots * prob.horizon * dynamics.dims(prob.dyn)[1]
    eps = noise.draw(prob.seed, prob.instance_id, kappa, i, prob.n_samples, D, samples)
    dev = sample_deformations(du_i, eps, ms[i], sg[i])
    u = effective_controls(prob, u_base, dev)
    x = dynamics.rollout(prob, x0, u)
    r, hits, robots_hit = fitness.reward(prob, x, goal)
    return dict(eps=eps, x=x, r=r, hits=hits, robots_hit=robots_hit)


def denoise_step(prob, x0, goal, u_base, du_i, kappa, i, eps=None, sched=None, pred_dtype=np.float64):
    """One step of Algorithm 1 at index i; returns a dict with every intermediate."""
    if sched is None:
        sched = schedule.step_scalars(prob.n_steps, prob.beta_min, prob.beta_max)
    ms, sg, os_ = sched
    D = prob.n_robots * prob.horizon * dynamics.dims(prob.dyn)[1]
    if eps is None:
        eps = noise.draw(prob.seed, prob.instance_id, kappa, i, prob.n_samples, D)
    samples = sample_deformations(du_i, eps, ms[i], sg[i])
    u = effective_controls(prob, u_base, samples)
    x = dynamics.rollout(prob, x0, u)
    r, hits, robots_hit = fitness.reward(prob, x, goal, pred_dtype)
    du_next, w = mc_update(du_i, eps, r, ms[i], sg[i], os_[i], prob.temperature,
                           bool(int(prob.flags) & FLAG_NORMALIZE))
    return dict(eps=eps, x=x, r=r, hits=hits, robots_hit=robots_hit, w=w, du_next=du_next)


def apply_deformation(prob, x0, goal, u_base, du0):
    """tau.u <- clip(tau.u + Delta U_0), then roll tau out (Algorithm 2 update)."""
    n, T, du = prob.n_robots, prob.horizon, dynamics.dims(prob.dyn)[1]
    u = dynamics.clip_controls(prob, np.asarray(u_base, dtype=np.float64).reshape(n, T, du)
                               + np.asarray(du0, dtype=np.float64).reshape(n, T, du))
    x = dynamics.rollout(prob, x0, u[None])
    r, hits, robots_hit = fitness.reward(prob, x, goal)
    return dict(u=u, x=x[0], r=float(r[0]), hits=int(hits[0]), robots_hit=int(robots_hit[0]),
                success=bool(fitness.success(prob, x, goal)[0]),
                at_goal=bool(fitness.at_goal(prob, x, goal)[0]),
                objective=float(fitness.objective(prob, x, goal)[0]))


def denoise_iteration(prob, x0, goal, u_base, kappa, trace=None):
    """One pass of Algorithm 2's loop body: Delta U_N = 0, steps N..1, then apply."""
    sched = schedule.step_scalars(prob.n_steps, prob.beta_min, prob.beta_max)
    D = prob.n_robots * prob.horizon * dynamics.dims(prob.dyn)[1]
    du = np.zeros(D)
    for i in range(prob.n_steps, 0, -1):
        out = denoise_step(prob, x0, goal, u_base, du, kappa, i, sched=sched)
        if trace is not None:
            trace.append(dict(i=i, du_in=du, **{k: out[k] for k in ("r", "hits", "w", "du_next")}))
        du = out["du_next"]
    res = apply_deformation(prob, x0, goal, u_base, du)
    res["du0"] = du
    return res


def plan(prob, x0, goal, iterations, u_init=None):
    """Algorithm 2 for a fixed number of iterations from zero controls (or u_init)."""
    n, T, du = prob.n_robots, prob.horizon, dynamics.dims(prob.dyn)[1]
    u = np.zeros((n, T, du)) if u_init is None else np.asarray(u_init, dtype=np.float64).reshape(n, T, du)
    history = []
    for kappa in range(iterations):
        res = denoise_iteration(prob, x0, goal, u, kappa)
        u = res["u"]
        history.append({k: res[k] for k in ("r", "hits", "success", "objective")})
    return u, history
