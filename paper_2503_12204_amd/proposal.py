"""Learned proposal: predict the initial plan of Algorithm 2 with a set network.

The paper starts every plan from an uninformed initialisation and lets the
deformation iterations of Algorithm 2 do all the work.  Here a
permutation-equivariant network (d4p_* in the C ABI, trained on the GPU by
this project's kernels) maps the start and goal sets of a team to an initial
plan tau.u; the plain planner then refines it exactly as before and also
judges it: the network's plan is kept only if its rolled-out reward beats the
zero plan's.

Training data are instances the plain planner itself solved (the batched
form labels hundreds at once).  The square workspace and the per-component
control box are invariant under the eight symmetries of the square, which
act on positions about the box centre and on the acceleration controls
alike, so every solved instance yields eight examples.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Sequence

import numpy as np
import torch

from . import workloads as W

# the eight symmetries of the square as 2x2 matrices
D4_MATS = [np.array(m, dtype=np.float64) for m in (
    [[1, 0], [0, 1]], [[0, -1], [1, 0]], [[-1, 0], [0, -1]], [[0, 1], [-1, 0]],
    [[-1, 0], [0, 1]], [[1, 0], [0, -1]], [[0, 1], [1, 0]], [[0, -1], [-1, 0]])]


def features(x0: np.ndarray, goal: np.ndarray, box: float) -> np.ndarray:
    """Per-robot inputs: start, goal and goal - start, centred and scaled by the half box."""
    c = box / 2.0
    s = np.asarray(x0, dtype=np.float64)[:, :2]
    g = np.asarray(goal, dtype=np.float64)[:, :2]
    return np.concatenate([(s - c) / c, (g - c) / c, (g - s) / c], axis=1).astype(np.float32)


def transform(x0, goal, u, mat, box):
    """Apply a symmetry of the square to starts, goals and the plan's accelerations."""
    c = box / 2.0
    x0 = np.asarray(x0, dtype=np.float64).copy()
    goal = np.asarray(goal, dtype=np.float64).copy()
    x0[:, :2] = c + (x0[:, :2] - c) @ mat.T
    x0[:, 2:4] = x0[:, 2:4] @ mat.T
    goal[:, :2] = c + (goal[:, :2] - c) @ mat.T
    u2 = None if u is None else np.asarray(u, dtype=np.float64) @ mat.T
    return x0.astype(np.float32), goal.astype(np.float32), (None if u2 is None else u2.astype(np.float32))


@dataclasses.dataclass
class Instance:
    prob: W.Problem
    x0: np.ndarray
    goal: np.ndarray


def random_team(rng, n_range=(4, 16), horizon=100, n_samples=2048, n_steps=100, box=10.0, min_sep=1.0,
                instance_id=0, seed=0) -> Instance:
    """2D holonomic team with random starts and goals in a box (the appendix's generic targets)."""
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    p, x0, g = W.random_instance(rng, W.HOLO2D, n, horizon, n_samples, box=box, min_sep=min_sep)
    p = p.replace(n_steps=n_steps, instance_id=instance_id, seed=seed)
    return Instance(p, x0, g)


def run_planner(L, insts: Sequence[Instance], iterations: int, init_plans=None, stop_all_success=False):
    """Algorithm 2 on many instances at once with the batched form.

    Returns (plans, per-iteration stats [K][count], seconds per iteration)."""
    bc = L.BatchContext([i.prob for i in insts], [i.x0 for i in insts], [i.goal for i in insts])
    try:
        if init_plans is not None:
            bc.set_plans(init_plans)
        hist = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(iterations):
            st = bc.iterate(k)
            hist.append(st)
            if stop_all_success and all(s["success"] for s in st):
                break
        dt = (time.perf_counter() - t0) / max(len(hist), 1)
        plans = [bc.plan_of(j).cpu().numpy() for j in range(len(insts))]
    finally:
        bc.close()
    return plans, hist, dt


def plan_reward(L, inst: Instance, plan) -> float:
    """Reward of a plan rolled out as is (the planner's judge of a proposal)."""
    p = inst.prob
    u = torch.as_tensor(np.asarray(plan, dtype=np.float32).reshape(1, p.n_robots, p.horizon, p.du), device="cuda")
    x = L.rollout(p, torch.as_tensor(inst.x0, device="cuda"), u)
    r, _, _ = L.fitness(p, x, torch.as_tensor(inst.goal, device="cuda"))
    return float(r.cpu()[0])


class Proposal:
    """The set network plus its feature pipeline."""

    def __init__(self, L, horizon=100, du=2, width=256, hidden=512, layers=4, max_rows=8192, max_batch=1024,
                 seed=0, box=10.0):
        self.L = L
        self.box = box
        self.horizon, self.du = horizon, du
        self.net = L.ProposalNet(d_in=6, width=width, hidden=hidden, layers=layers, d_out=horizon * du,
                                 max_rows=max_rows, max_batch=max_batch, seed=seed)

    def _pack(self, xs: List[np.ndarray]):
        seg = np.concatenate([[0], np.cumsum([x.shape[0] for x in xs])]).astype(np.int32)
        return torch.as_tensor(np.concatenate(xs), device="cuda"), torch.as_tensor(seg, device="cuda"), seg

    def fit(self, insts: Sequence[Instance], plans, mask, epochs=20, batch=64, lr=1e-3, augment=True, seed=0,
            log=None):
        """Adam on the masked MSE between predicted and solved plans (cosine-decayed rate)."""
        rng = np.random.default_rng(seed)
        ex_x, ex_t, ex_m = [], [], []
        mats = D4_MATS if augment else D4_MATS[:1]
        for inst, plan, mk in zip(insts, plans, mask):
            for mat in mats:
                x0, g, u = transform(inst.x0, inst.goal, plan, mat, self.box)
                ex_x.append(features(x0, g, self.box))
                ex_t.append(u.reshape(inst.prob.n_robots, -1))
                ex_m.append(np.full(inst.prob.n_robots, float(mk), dtype=np.float32))
        n_ex = len(ex_x)
        steps = epochs * max(1, n_ex // batch)
        losses = []
        k = 0
        for ep in range(epochs):
            order = rng.permutation(n_ex)
            for b0 in range(0, n_ex - batch + 1, batch):
                idx = order[b0:b0 + batch]
                x, seg_t, _ = self._pack([ex_x[i] for i in idx])
                t = torch.as_tensor(np.concatenate([ex_t[i] for i in idx]), device="cuda")
                m = torch.as_tensor(np.concatenate([ex_m[i] for i in idx]), device="cuda")
                rate = lr * 0.5 * (1 + np.cos(np.pi * k / max(steps, 1)))
                loss = self.net.train_step(x, seg_t, t, m, max(rate, 1e-6))
                k += 1
            losses.append(float(loss.cpu()))
            if log:
                log(f"epoch {ep} loss {losses[-1]:.5f}")
        return losses

    def predict(self, insts: Sequence[Instance]):
        """Predicted plans, clipped to the control box."""
        out = []
        for c0 in range(0, len(insts), 256):
            chunk = insts[c0:c0 + 256]
            x, seg_t, seg = self._pack([features(i.x0, i.goal, self.box) for i in chunk])
            y = self.net.forward(x, seg_t).cpu().numpy()
            for j, inst in enumerate(chunk):
                p = inst.prob
                lo, hi = np.array(p.u_lo[:p.du]), np.array(p.u_hi[:p.du])
                u = y[seg[j]:seg[j + 1]].reshape(p.n_robots, p.horizon, p.du)
                out.append(np.clip(u, lo, hi).astype(np.float32))
        return out

    def judged_initial_plans(self, insts: Sequence[Instance]):
        """The network's plan where its reward beats the zero plan's, else the zero plan."""
        preds = self.predict(insts)
        plans, used = [], []
        for inst, u in zip(insts, preds):
            zero = np.zeros_like(u)
            if plan_reward(self.L, inst, u) > plan_reward(self.L, inst, zero):
                plans.append(u)
                used.append(True)
            else:
                plans.append(zero)
                used.append(False)
        return plans, used

    def close(self):
        self.net.close()


def iterations_to_target(hist, target, init_rewards=None):
    """First iteration count (0 = the initial plan) whose reward reaches each target."""
    K = len(hist)
    out = []
    for j, tj in enumerate(target):
        k_hit = K + 1
        if init_rewards is not None and init_rewards[j] >= tj:
            k_hit = 0
        else:
            for k in range(K):
                if hist[k][j]["reward"] >= tj:
                    k_hit = k + 1
                    break
        out.append(k_hit)
    return np.array(out)
