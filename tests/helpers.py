"""Shared test helpers: tolerances, guard bands and problem builders."""
import numpy as np

from paper_2503_12204_amd import workloads as W

# Single RK4 step, FP32 kernel vs FP64 oracle from the same FP32 state:
# a handful of roundings of |x| plus the hardware sine/cosine error.
STEP_RTOL, STEP_ATOL = 1e-5, 1e-6
# Per-sample reward: each r_goal term carries the position error of its
# step (below 1e-4 m over 160 FP32 steps) times 1/d0 (<= 10) and an FP32
# sqrt/division; the average over n*T terms keeps that bound.
REWARD_ATOL = 2e-4
# Final reward of an iteration, relative (the stated bar is 1e-3).
FINAL_RTOL = 1e-3
# A pair whose FP64 squared distance lies within this fraction of the squared
# threshold may legitimately be judged differently on FP32 positions: an FP32
# rollout of T <= 160 steps keeps positions within ~1e-4 m of FP64, which moves
# a squared distance near the 0.7 m threshold by at most ~4 * 0.7 * 1e-4.
GUARD_BAND = 6e-4


def ambiguous_samples(prob, x, band=GUARD_BAND):
    """Samples with any pair, any step, inside the guard band of the reward threshold."""
    dp = W.dims(prob.dyn)[2]
    pos = np.moveaxis(np.asarray(x, dtype=np.float64)[:, :, 1:, :dp], 2, 1)  # [M, T, n, dp]
    d = pos[:, :, :, None, :] - pos[:, :, None, :, :]
    d2 = (d ** 2).sum(-1)
    thr = 2 * float(np.float32(prob.robot_radius)) + float(np.float32(prob.safety_margin))
    near = np.abs(d2 - thr * thr) <= band * thr * thr
    n = x.shape[1]
    near &= ~np.eye(n, dtype=bool)
    return near.any(axis=(1, 2, 3))


def ambiguous_obstacle_samples(prob, x, band=GUARD_BAND):
    """Samples with a state inside the guard band of an obstacle's reward distance."""
    dp = W.dims(prob.dyn)[2]
    obs = np.asarray(prob.obstacles, dtype=np.float32).reshape(-1, 4).astype(np.float64)
    M = np.asarray(x).shape[0]
    if len(obs) == 0:
        return np.zeros(M, dtype=bool)
    pos = np.asarray(x, dtype=np.float64)[:, :, 1:, :dp]
    d2 = ((pos[..., None, :] - obs[:, :dp]) ** 2).sum(-1)                    # [M, n, T, O]
    thr = float(np.float32(prob.robot_radius)) + obs[:, 3] + float(np.float32(prob.safety_margin))
    return (np.abs(d2 - thr * thr) <= band * thr * thr).any(axis=(1, 2, 3))


def ambiguous_band_pairs(prob, x, band=GUARD_BAND):
    """Per sample, the number of (pair, step) checks inside the guard band."""
    dp = W.dims(prob.dyn)[2]
    pos = np.moveaxis(np.asarray(x, dtype=np.float64)[:, :, 1:, :dp], 2, 1)
    d = pos[:, :, :, None, :] - pos[:, :, None, :, :]
    d2 = (d ** 2).sum(-1)
    thr = 2 * float(np.float32(prob.robot_radius)) + float(np.float32(prob.safety_margin))
    near = np.abs(d2 - thr * thr) <= band * thr * thr
    near = np.triu(near, k=1)
    return near.sum(axis=(1, 2, 3))


def problems_small():
    """Parity shapes: several tiles with a ragged tail, odd horizons, edge team sizes."""
    out = []
    p, x0, g = W.holo2d_circle(n=4, horizon=50, n_samples=300)
    out.append(("holo2d_n4_T50_M300", p, x0, g))
    rng = np.random.default_rng(11)
    p, x0, g = W.random_instance(rng, W.HOLO3D, 16, 37, 100, box=4.0, min_sep=0.8)
    out.append(("holo3d_n16_T37_M100", p, x0, g))
    p, x0, g = W.unicycle_random(n=8, horizon=60, n_samples=257, box=5.0, min_sep=0.8, instance_seed=3)
    out.append(("unicycle_n8_T60_M257", p, x0, g))
    p, x0, g = W.random_instance(rng, W.HOLO2D, 5, 13, 70, box=3.0, min_sep=0.7)
    out.append(("holo2d_n5_T13_M70", p, x0, g))
    p, x0, g = W.random_instance(rng, W.UNICYCLE, 3, 41, 64, box=3.0, min_sep=0.7)
    out.append(("unicycle_n3_T41_M64", p, x0, g))
    p, x0, g = W.random_instance(rng, W.HOLO2D, 32, 20, 48, box=6.0, min_sep=0.6)
    out.append(("holo2d_n32_T20_M48", p, x0, g))
    p, x0, g = W.random_instance(rng, W.HOLO3D, 1, 9, 33, box=3.0)
    out.append(("holo3d_n1_T9_M33", p, x0, g))
    p, x0, g = W.random_instance(rng, W.UNICYCLE, 2, 1, 1, box=3.0)
    out.append(("unicycle_n2_T1_M1", p, x0, g))
    p, x0, g = W.diffdrive_circle(n=6, horizon=33, n_samples=130, radius=1.5)
    out.append(("diffdrive_n6_T33_M130", p, x0, g))
    p, x0, g = W.random_instance(rng, W.DIFFDRIVE, 11, 24, 96, box=4.0, min_sep=0.7)
    out.append(("diffdrive_n11_T24_M96", p, x0, g))
    p, x0, g = W.holo2d_circle_obstacles(n=8, n_obs=3, horizon=40, n_samples=200)
    out.append(("holo2d_obs3_n8_T40_M200", p, x0, g))
    p, x0, g = W.random_instance(rng, W.HOLO3D, 6, 30, 90, box=3.0, min_sep=0.7,
                                 obstacles=((1.5, 1.5, 1.5, 0.5), (0.5, 2.5, 1.0, 0.3)))
    out.append(("holo3d_obs2_n6_T30_M90", p, x0, g))
    # the longest horizon of the batched workloads (160 steps): the heading of
    # the unicycle and of the differential drive is not wrapped, so late steps
    # take sines and cosines of angles up to |omega| T dt = 16 pi
    p, x0, g = W.random_instance(rng, W.UNICYCLE, 8, 160, 128, box=6.0, min_sep=0.8)
    out.append(("unicycle_n8_T160_M128", p, x0, g))
    p, x0, g = W.random_instance(rng, W.DIFFDRIVE, 12, 160, 96, box=6.0, min_sep=0.8)
    out.append(("diffdrive_n12_T160_M96", p, x0, g))
    return out
