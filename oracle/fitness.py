"""Team reward, success and objective (Sections III and IV-A).

Eq. generic-reward: r(tau) = 1/(n H) sum_{t=1..H} sum_k (r_goal(k, t) + w_t r_safe(k, t)),
with r_goal(k, t) = 1 - |p_k[t] - g_k| / |p_k[start] - g_k| and r_safe(k, t) = -1
when robot k is within 2 R_a + epsilon of some other robot l at time t, else 0.

Readings (the paper is ambiguous or silent):
* T controls give T + 1 states x[0..T]; sums run over x[1..T], the r_goal
  denominator uses x[0] and is floored at d0_floor (start = goal gives 0/0).
* r_safe is binary per robot and step ("any" partner); with the SAFE_PAIRS
  flag it is minus the number of partners instead.
* w_t is a constant w_safe.
* hits counts colliding pairs k < l summed over t = 1..T (an integer).
* The pair predicate is |p_k - p_l|^2 <= thr2 with thr2 = (2 R_a + epsilon)^2.
  When it is evaluated on FP32 positions the squared distance is formed in
  FP32 as ((dx*dx + dy*dy) + dz*dz), each operation rounded, and thr2 is the
  FP32 rounding of the FP64 square; on FP64 positions everything is FP64.
* success: every pair strictly farther apart than 2 R_a at t = 1..T (the safety
  condition); Section V-A glosses a successful solution as feasible and
  conflict-free, and feasibility holds by construction of the rollout.
* at_goal: every robot within goal_tol of its goal at t = T (the terminal
  condition read with a tolerance), reported beside success.
* objective (Eq. objective): fraction of robot-steps t = 1..T within goal_tol.
* Obstacles (appendix, "a binary penalty term for whether the robot collides
  with any obstacle" added to Eq. generic-reward): r_obs(k, t) = -1 when robot
  k is within R_a + r_o + epsilon of some obstacle o, weighted like r_safe
  (w_safe); the predicate is |p_k - c_o|^2 <= (R_a + r_o + epsilon)^2, formed
  like the pair predicate.  Success also requires every state strictly
  farther than R_a + r_o from every obstacle.

Pinned by brute-force pair loops on small teams, a closed-form head-on pass,
closed-form rewards of stationary teams and permutation invariance
(tests/test_oracle_fitness.py).
"""
import numpy as np

from .dynamics import dims

FLAG_NORMALIZE = 1
FLAG_SAFE_PAIRS = 2


def threshold_sq(prob, dtype):
    """Squared reward safety distance (2 R_a + epsilon)^2 in the given dtype."""
    thr = 2.0 * float(np.float32(prob.robot_radius)) + float(np.float32(prob.safety_margin))
    return dtype(thr * thr)


def pair_dist_sq(pos, dtype):
    """|p_k - p_l|^2 for all k, l; pos [..., n, d_p] -> [..., n, n] in dtype."""
    p = np.asarray(pos).astype(dtype)
    d = p[..., :, None, :] - p[..., None, :, :]
    acc = d[..., 0] * d[..., 0]
    for c in range(1, p.shape[-1]):
        acc = acc + d[..., c] * d[..., c]
    return acc


def _obstacles(prob, dp):
    """(centres [O][d_p], radii [O]) of the problem's obstacles, FP32-rounded."""
    obs = np.asarray(prob.obstacles, dtype=np.float32).reshape(-1, 4)
    return obs[:, :dp].astype(np.float64), obs[:, 3].astype(np.float64)


def obstacle_dist_sq(pos, centres, dtype):
    """|p - c_o|^2 for every obstacle; pos [..., d_p] -> [..., O] in dtype,
    in the pair predicate's order ((dx*dx + dy*dy) + dz*dz)."""
    p = np.asarray(pos).astype(dtype)[..., None, :]
    d = p - np.asarray(centres).astype(dtype)
    acc = d[..., 0] * d[..., 0]
    for c in range(1, d.shape[-1]):
        acc = acc + d[..., c] * d[..., c]
    return acc


def obstacle_hits(prob, x, pred_dtype=np.float64):
    """[M, n, T] bool: the state at t = 1..T is within R_a + r_o + epsilon of some obstacle."""
    _, _, dp = dims(prob.dyn)
    x = np.asarray(x)
    M, n, T1, _ = x.shape
    cen, rad = _obstacles(prob, dp)
    if len(rad) == 0:
        return np.zeros((M, n, T1 - 1), dtype=bool)
    ra = float(np.float32(prob.robot_radius))
    eps = float(np.float32(prob.safety_margin))
    thr = (ra + rad + eps) ** 2
    d2 = obstacle_dist_sq(x[:, :, 1:, :dp], cen, pred_dtype)          # [M, n, T, O]
    return (d2 <= thr.astype(pred_dtype)).any(axis=-1)


def reward(prob, x, goal, pred_dtype=np.float64):
    """(r [M], hits [M], robots_hit [M]) for trajectories x [M][n][T+1][d_x].

    robots_hit counts robot-steps with r_safe != 0.  pred_dtype selects the
    precision of the pair predicate (np.float32 when x holds FP32 positions
    that must be judged exactly as the FP32 path judges them).
    """
    _, _, dp = dims(prob.dyn)
    x = np.asarray(x)
    M, n, T1, _ = x.shape
    T = T1 - 1
    pos = x[..., :dp]
    g = np.asarray(goal, dtype=np.float64)[None, :, :]
    pos64 = pos.astype(np.float64)
    d0 = np.linalg.norm(pos64[:, :, 0, :] - g, axis=-1)              # [M, n]
    d0 = np.maximum(d0, float(np.float32(prob.d0_floor)))
    dist = np.linalg.norm(pos64[:, :, 1:, :] - g[:, :, None, :], axis=-1)  # [M, n, T]
    r_goal = 1.0 - dist / d0[:, :, None]
    # pair predicate per step
    pt = np.moveaxis(pos[:, :, 1:, :], 2, 1)                          # [M, T, n, dp]
    d2 = pair_dist_sq(pt, pred_dtype)                                 # [M, T, n, n]
    hit = d2 <= threshold_sq(prob, pred_dtype)
    eye = np.eye(n, dtype=bool)
    hit &= ~eye
    partners = hit.sum(axis=-1)                                       # [M, T, n]
    if int(prob.flags) & FLAG_SAFE_PAIRS:
        r_safe = -partners.astype(np.float64)
    else:
        r_safe = -(partners > 0).astype(np.float64)
    r_safe = np.moveaxis(r_safe, 1, 2)                                # [M, n, T]
    r_obs = -obstacle_hits(prob, x, pred_dtype).astype(np.float64)   # [M, n, T]
    w = float(np.float32(prob.w_safe))
    r = (r_goal + w * (r_safe + r_obs)).sum(axis=(1, 2)) / (n * T)
    hits = np.triu(hit, k=1).sum(axis=(1, 2, 3)).astype(np.int64)
    robots_hit = (partners > 0).sum(axis=(1, 2)).astype(np.int64)
    return r, hits, robots_hit


def success(prob, x, goal):
    """Safety at t = 1..T: every pair strictly farther apart than 2 R_a."""
    _, _, dp = dims(prob.dyn)
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[1]
    pos = x[..., 1:, :dp]                                             # [M, n, T, dp]
    pt = np.moveaxis(pos, 2, 1)
    d = np.sqrt(pair_dist_sq(pt, np.float64))
    d = d + np.eye(n) * 1e30
    safe = (d > 2.0 * float(np.float32(prob.robot_radius))).all(axis=(1, 2, 3))
    cen, rad = _obstacles(prob, dp)
    if len(rad):
        do = np.sqrt(obstacle_dist_sq(pos, cen, np.float64))              # [M, n, T, O]
        safe &= (do > float(np.float32(prob.robot_radius)) + rad).all(axis=(1, 2, 3))
    return safe


def at_goal(prob, x, goal):
    """Terminal condition: every robot within goal_tol of its goal at t = T."""
    _, _, dp = dims(prob.dyn)
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(goal, dtype=np.float64)[None, :, :]
    return (np.linalg.norm(x[:, :, -1, :dp] - g, axis=-1) <= float(np.float32(prob.goal_tol))).all(axis=1)


def objective(prob, x, goal):
    """Fraction of robot-steps (t = 1..T) within goal_tol of the goal."""
    _, _, dp = dims(prob.dyn)
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(goal, dtype=np.float64)[None, :, None, :]
    at = np.linalg.norm(x[:, :, 1:, :dp] - g, axis=-1) <= float(np.float32(prob.goal_tol))
    n, T = x.shape[1], x.shape[2] - 1
    return at.sum(axis=(1, 2)) / (n * T)
