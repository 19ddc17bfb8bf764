"""Problem records and seeded synthetic instance generators.

This module holds no arithmetic of the planning method itself: it only
describes a planning problem (Section III of the paper: team size, dynamics,
horizon, time step, robot radius, start and goal states) together with the
sampler and schedule settings of Algorithm 1, and draws start/goal sets of the
shapes the paper evaluates (antipodal circle and sphere swaps, Section V-A;
random start and goal sets in a square, the generic target assignment study of
the appendix).  Both the HIP path and the CPU checker consume what it makes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

HOLO2D = 0
HOLO3D = 1
UNICYCLE = 2
DIFFDRIVE = 3
DYN_NAMES = {HOLO2D: "holo2d", HOLO3D: "holo3d", UNICYCLE: "unicycle", DIFFDRIVE: "diffdrive"}

# flag bits (same values as the C header)
FLAG_NORMALIZE = 1     # z-score the rewards of one batch before the softmax
FLAG_SAFE_PAIRS = 2    # r_safe counts every colliding partner instead of "any"


def dims(dyn: int) -> Tuple[int, int, int]:
    """(state dim, control dim, position dim) of a dynamics id."""
    if dyn == HOLO2D:
        return 4, 2, 2
    if dyn == HOLO3D:
        return 6, 3, 3
    if dyn == UNICYCLE:
        return 3, 2, 2
    if dyn == DIFFDRIVE:
        return 4, 2, 2
    raise ValueError(f"unknown dynamics id {dyn}")


@dataclasses.dataclass
class Problem:
    """One planning problem plus sampler settings (mirrors ``d4_problem``)."""
    dyn: int = HOLO2D
    n_robots: int = 4
    horizon: int = 50           # T: controls u[0..T-1], states x[0..T]
    n_samples: int = 256        # M Monte Carlo samples per denoising step
    n_steps: int = 100          # N denoising steps per iteration
    dt: float = 0.1
    robot_radius: float = 0.3   # R_a
    safety_margin: float = 0.1  # epsilon in r_safe
    w_safe: float = 1.0         # weight of r_safe in the team reward
    temperature: float = 0.1    # lambda
    beta_min: float = 1e-4
    beta_max: float = 1e-2
    u_lo: Tuple[float, float, float] = (-1.0, -1.0, -1.0)
    u_hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    v_max: float = 2.0          # per-component speed bound (holonomic)
    goal_tol: float = 0.1       # terminal-condition tolerance
    d0_floor: float = 0.1       # floor of the r_goal denominator
    flags: int = FLAG_NORMALIZE
    instance_id: int = 0
    seed: int = 0
    # static obstacles (appendix): (x, y, z, radius) each, z unused in 2D
    obstacles: Tuple[Tuple[float, float, float, float], ...] = ()

    @property
    def dx(self) -> int:
        return dims(self.dyn)[0]

    @property
    def du(self) -> int:
        return dims(self.dyn)[1]

    @property
    def dp(self) -> int:
        return dims(self.dyn)[2]

    @property
    def D(self) -> int:
        """Length of one joint deformation vector, n * T * d_u."""
        return self.n_robots * self.horizon * self.du

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------- geometry
def circle_swap(n: int, radius: float = 2.0) -> Tuple[np.ndarray, np.ndarray]:
    """n points evenly on a circle, each heading to its antipode."""
    ang = 2.0 * np.pi * np.arange(n) / n
    start = np.stack([radius * np.cos(ang), radius * np.sin(ang)], axis=1)
    return start, -start


def sphere_swap(n: int, radius: float = 2.0) -> Tuple[np.ndarray, np.ndarray]:
    """n points on a sphere (Fibonacci lattice), each heading to its antipode."""
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    rr = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.pi * (3.0 - np.sqrt(5.0)) * i
    start = radius * np.stack([rr * np.cos(phi), rr * np.sin(phi), z], axis=1)
    return start, -start


def random_points(rng: np.random.Generator, n: int, dp: int, box: float,
                  min_sep: float, max_tries: int = 10000) -> np.ndarray:
    """n points uniform in [0, box]^dp with pairwise separation >= min_sep."""
    pts: List[np.ndarray] = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries * n:
            raise RuntimeError("could not place points with the requested separation")
        p = rng.uniform(0.0, box, size=dp)
        if all(np.linalg.norm(p - q) >= min_sep for q in pts):
            pts.append(p)
    return np.array(pts)


def make_states(dyn: int, start_pos: np.ndarray, goal_pos: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Full start states (velocity 0; unicycle and differential drive heading
    toward the goal) and goal positions."""
    dx, _, dp = dims(dyn)
    n = start_pos.shape[0]
    x0 = np.zeros((n, dx), dtype=np.float64)
    x0[:, :dp] = start_pos
    if dyn in (UNICYCLE, DIFFDRIVE):
        d = goal_pos - start_pos
        x0[:, 2] = np.arctan2(d[:, 1], d[:, 0])
    return x0.astype(np.float32), goal_pos.astype(np.float32)


# ------------------------------------------------------ named workloads
def holo2d_circle(n: int = 4, horizon: int = 50, n_samples: int = 256, radius: float = 2.0,
                  **kw) -> Tuple[Problem, np.ndarray, np.ndarray]:
    """2D holonomic antipodal circle swap (4 robots, T=50, M=256 by default)."""
    p = Problem(dyn=HOLO2D, n_robots=n, horizon=horizon, n_samples=n_samples,
                u_lo=(-1.0, -1.0, -1.0), u_hi=(1.0, 1.0, 1.0), v_max=2.0, **kw)
    s, g = circle_swap(n, radius)
    x0, goal = make_states(HOLO2D, s, g)
    return p, x0, goal


def unicycle_random(n: int = 8, horizon: int = 100, n_samples: int = 2048, box: float = 10.0,
                    min_sep: float = 1.0, instance_seed: int = 0,
                    **kw) -> Tuple[Problem, np.ndarray, np.ndarray]:
    """Unicycle team with random start and goal sets in a box (8 robots, T=100, M=2048)."""
    rng = np.random.default_rng(instance_seed)
    s = random_points(rng, n, 2, box, min_sep)
    g = random_points(rng, n, 2, box, min_sep)
    p = Problem(dyn=UNICYCLE, n_robots=n, horizon=horizon, n_samples=n_samples,
                u_lo=(-1.0, -math.pi, 0.0), u_hi=(1.0, math.pi, 0.0), v_max=0.0, **kw)
    x0, goal = make_states(UNICYCLE, s, g)
    return p, x0, goal


# differential drive (Section V model): turn rate within +-pi rad/s, tangential
# acceleration within +-1 m/s^2, speed within +-1 m/s (the unicycle's speed bound)
DIFFDRIVE_LIMITS = dict(u_lo=(-math.pi, -1.0, 0.0), u_hi=(math.pi, 1.0, 0.0), v_max=1.0)


def diffdrive_circle(n: int = 8, horizon: int = 100, n_samples: int = 2048, radius: float = 2.0,
                     **kw) -> Tuple[Problem, np.ndarray, np.ndarray]:
    """Differential-drive antipodal circle swap (Section V-A scenario with the
    paper's own differential-drive model)."""
    s, g = circle_swap(n, radius)
    lim = DIFFDRIVE_LIMITS.copy()
    lim.update(kw)
    p = Problem(dyn=DIFFDRIVE, n_robots=n, horizon=horizon, n_samples=n_samples, **lim)
    x0, goal = make_states(DIFFDRIVE, s, g)
    return p, x0, goal


def circle_obstacles(n_obs: int, ring: float = 0.8, big: float = 0.6,
                     small: float = 0.3) -> Tuple[Tuple[float, float, float, float], ...]:
    """Obstacles for the antipodal swap with obstacles (appendix): one large
    disc at the centre, or n_obs small discs evenly on a ring around it."""
    if n_obs <= 0:
        return ()
    if n_obs == 1:
        return ((0.0, 0.0, 0.0, big),)
    ang = 2.0 * np.pi * np.arange(n_obs) / n_obs + 0.25
    return tuple((float(ring * np.cos(a)), float(ring * np.sin(a)), 0.0, small) for a in ang)


def holo2d_circle_obstacles(n: int = 16, n_obs: int = 4, horizon: int = 100, n_samples: int = 2048,
                            radius: float = 2.0, **kw) -> Tuple[Problem, np.ndarray, np.ndarray]:
    """2D holonomic antipodal circle swap around static obstacles (appendix scenario)."""
    s, g = circle_swap(n, radius)
    p = Problem(dyn=HOLO2D, n_robots=n, horizon=horizon, n_samples=n_samples,
                u_lo=(-1.0, -1.0, -1.0), u_hi=(1.0, 1.0, 1.0), v_max=2.0,
                obstacles=circle_obstacles(n_obs), **kw)
    x0, goal = make_states(HOLO2D, s, g)
    return p, x0, goal


def holo3d_sphere(n: int = 16, horizon: int = 100, n_samples: int = 8192, radius: float = 2.0,
                  **kw) -> Tuple[Problem, np.ndarray, np.ndarray]:
    """3D holonomic antipodal sphere swap (16 robots, T=100, M=8192)."""
    p = Problem(dyn=HOLO3D, n_robots=n, horizon=horizon, n_samples=n_samples,
                u_lo=(-1.0, -1.0, -1.0), u_hi=(1.0, 1.0, 1.0), v_max=2.0, **kw)
    s, g = sphere_swap(n, radius)
    x0, goal = make_states(HOLO3D, s, g)
    return p, x0, goal


def random_instance(rng: np.random.Generator, dyn: int, n: int, horizon: int, n_samples: int,
                    box: float = 10.0, min_sep: float = 1.0,
                    **kw) -> Tuple[Problem, np.ndarray, np.ndarray]:
    """Random start/goal instance of any dynamics in a box (cube in 3D)."""
    _, _, dp = dims(dyn)
    s = random_points(rng, n, dp, box, min_sep)
    g = random_points(rng, n, dp, box, min_sep)
    if dyn == UNICYCLE:
        lim = dict(u_lo=(-1.0, -math.pi, 0.0), u_hi=(1.0, math.pi, 0.0), v_max=0.0)
    elif dyn == DIFFDRIVE:
        lim = DIFFDRIVE_LIMITS.copy()
    else:
        lim = dict(u_lo=(-1.0, -1.0, -1.0), u_hi=(1.0, 1.0, 1.0), v_max=2.0)
    lim.update(kw)
    p = Problem(dyn=dyn, n_robots=n, horizon=horizon, n_samples=n_samples, **lim)
    x0, goal = make_states(dyn, s, g)
    return p, x0, goal


def batched_mix(count: int = 512, n_samples: int = 1024, n_range=(2, 32), t_range=(40, 160),
                seed: int = 0, box: float = 10.0):
    """Uneven batch: robots ~ U{2..32}, horizon ~ U{40..160}, dynamics ~ U{3 kinds}."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        dyn = int(rng.integers(0, 3))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        T = int(rng.integers(t_range[0], t_range[1] + 1))
        # a 10 m box holds 32 robots at 1 m separation easily in 2D and 3D
        p, x0, goal = random_instance(rng, dyn, n, T, n_samples, box=box)
        out.append((p.replace(instance_id=j), x0, goal))
    return out
