"""Time-to-target comparisons of the batched and learned-proposal forms
against the plain planner on the same GPU.

batched_vs_plain: many uneven instances, one batched iteration against the
    same instances run one after another through the single-problem path
    (identical results, so time-to-target is the time for the same work).
proposal_gain: train the proposal on teams the planner solved, then run the
    plain planner from zero controls and from the judged proposal on
    held-out teams; an instance's target is 99.5 % of the reward the plain
    planner reaches with its full iteration budget (the budget's reward
    itself is reported as the strict target).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import proposal as PR
from . import workloads as W


def algorithmic_ops(dyn, n, n_obstacles=0):
    """The method's VALU operations per robot*step*sample (draws, sampled
    control, dynamics, goal term and the pair term of Eq. generic-reward with
    (n - 1)/2 checks per robot and step): the numerator of the fused kernels'
    roofline."""
    dx, du, dp = W.dims(dyn)
    dynamics = 80.0 if dyn in (W.UNICYCLE, W.DIFFDRIVE) else 5.0 * dp
    check = 2.0 * dp + 2.0
    return 40.0 * du + 3.0 * du + dynamics + 8.0 + (n - 1) / 2.0 * check + n_obstacles * check


def _time_batch(L, inst, iterations):
    probs = [p for p, _, _ in inst]
    bc = L.BatchContext(probs, [x for _, x, _ in inst], [g for _, _, g in inst])
    bc.iterate(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(iterations):
        bc.iterate(k + 1, sync=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iterations
    bc.close()
    return dt


def batched_vs_plain(L, count=512, n_samples=1024, iterations=2, seed=0, plain=True, tune=True, log=print):
    """The batched form against the same instances run one after another
    through the single-problem path.  With tune, the batch's bucket tiles are
    also chosen by coordinate descent on the time of short whole-batch
    iterations (autotune.tune_batch, starting from the rule; the tuning time
    is reported, not counted), and the batch is timed with them."""
    from . import autotune as AT
    inst = W.batched_mix(count=count, n_samples=n_samples, seed=seed)
    probs = [p for p, _, _ in inst]
    units = sum(p.n_robots * p.horizon * p.n_samples * p.n_steps for p in probs)
    ops_per_step = sum(algorithmic_ops(p.dyn, p.n_robots, len(p.obstacles)) * p.n_robots * p.horizon * p.n_samples
                       for p in probs)
    t_rule = _time_batch(L, inst, iterations)
    log(f"batched, rule tiles: {t_rule * 1e3:.1f} ms per iteration of {count} instances")
    tuned = None
    t_batch = t_rule
    if tune:
        import tempfile
        t0 = time.perf_counter()
        with tempfile.TemporaryDirectory() as td:
            tuned = AT.tune_batch(probs, [x for _, x, _ in inst], [g for _, _, g in inst],
                                  path=f"{td}/tiles.json", log=log)
        t_tune = time.perf_counter() - t0
        t_batch = _time_batch(L, inst, iterations)
        for b in {AT.batch_bucket(p) for p in probs}:
            AT.clear_batch_tile(b)
        log(f"batched, tuned tiles ({t_tune:.1f} s of tuning): {t_batch * 1e3:.1f} ms per iteration")
    head = {"instances": count, "samples": n_samples, "batched_ms_per_iteration": t_batch * 1e3,
            "batched_rule_tiles_ms_per_iteration": t_rule * 1e3,
            "tuned_tiles": {"/".join(str(v) for v in b): e for b, e in tuned.items()} if tuned is not None else None,
            "batched_robot_step_samples_per_s": units / t_batch, "algorithmic_ops_per_step": ops_per_step,
            "step_algorithmic_rate_T_per_s": ops_per_step * probs[0].n_steps / t_batch / 1e12}
    if not plain:
        return head
    ctxs = []
    for p, x0, g in inst:
        ctxs.append((L.Context(p), torch.as_tensor(x0, device="cuda"), torch.as_tensor(g, device="cuda"),
                     torch.zeros((p.n_robots, p.horizon, p.du), device="cuda")))
    for c, x0, g, u in ctxs:
        c.denoise_iter(x0, g, u, 0, sync=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(iterations):
        for c, x0, g, u in ctxs:
            c.denoise_iter(x0, g, u, k + 1, sync=False)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / iterations
    for c, _, _, _ in ctxs:
        c.close()
    log(f"plain, one instance after another: {t_plain * 1e3:.1f} ms per iteration")
    head.update({"plain_sequential_ms_per_iteration": t_plain * 1e3, "speedup": t_plain / t_batch})
    return head


def _chunks(seq, k):
    for i in range(0, len(seq), k):
        yield seq[i:i + k]


def proposal_gain(L, n_train=4096, n_test=1000, label_samples=1024, label_iters=3, eval_samples=2048,
                  eval_iters=5, extra_iters=3, epochs=20, seed=0, target_tol=0.005, log=print):
    """Train the proposal on teams the plain planner solved, then compare the
    plain planner from zero controls with the planner started from the judged
    proposal on held-out teams.

    An instance's target is 99.5 % of the reward the plain planner reaches with
    its budget of eval_iters iterations (the strict target, that reward itself,
    is reported too).  The proposal-started run gets extra_iters iterations
    beyond the budget, so that a team it misses is a team it does not reach in
    eval_iters + extra_iters iterations; the miss fraction, the speedup over
    the teams both runs reach, and the speedup with each miss counted at the
    cap are all reported.  Two judges decide which start a team keeps:
      initial: the proposal when its rolled-out reward beats the zero plan's
               (the planner's fitness of the initial plans, no extra cost);
      first iteration: the start whose reward after one iteration is higher,
               which costs one extra iteration per team (counted) and guards
               the final quality as well as the start.
    The fraction of teams whose reward after the budget ends below the plain
    planner's is reported for each."""
    rng = np.random.default_rng(1_000_000 + seed)
    t0 = time.perf_counter()
    train = []
    for j in range(n_train):
        train.append(PR.random_team(rng, n_samples=label_samples, instance_id=j))
        if (j + 1) % 20000 == 0:
            log(f"built {j + 1} training teams")
    plans, rewards, success = [], [], []
    for c, chunk in enumerate(_chunks(train, 512)):
        pl, hist, _ = PR.run_planner(L, chunk, iterations=label_iters)
        plans += pl
        rewards += [s["reward"] for s in hist[-1]]
        success += [s["success"] for s in hist[-1]]
        if (c + 1) % 20 == 0:
            log(f"labelled {len(plans)} teams, {time.perf_counter() - t0:.0f} s")
    rewards, success = np.array(rewards), np.array(success)
    mask = success if success.mean() >= 0.25 else rewards >= np.median(rewards)
    t_label = time.perf_counter() - t0
    log(f"labelled {n_train} teams in {t_label:.1f} s: success {success.mean():.3f}, "
        f"mean reward {rewards.mean():.4f}, training on {int(mask.sum())}")
    prop = PR.Proposal(L, seed=seed)
    t0 = time.perf_counter()
    losses = prop.fit(train, plans, mask, epochs=epochs, batch=64, lr=1e-3, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained {epochs} epochs in {t_train:.1f} s, loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    del train, plans

    trng = np.random.default_rng(seed)
    test = [PR.random_team(trng, n_samples=eval_samples, instance_id=j) for j in range(n_test)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    init, used = prop.judged_initial_plans(test)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    r_init = np.array([PR.plan_reward(L, t, u) for t, u in zip(test, init)])
    hp, hn, tp = [], [], []
    K_n = eval_iters + extra_iters
    for c0 in range(0, n_test, 500):
        ch = test[c0:c0 + 500]
        _, h1, t1 = PR.run_planner(L, ch, iterations=eval_iters)
        _, h2, _ = PR.run_planner(L, ch, iterations=K_n, init_plans=init[c0:c0 + 500])
        hp.append(h1)
        hn.append(h2)
        tp.append(t1)                # seconds per batched iteration of this chunk
        log(f"evaluated {c0 + len(ch)} held-out teams")
    hist_p = [sum((h[k] for h in hp), []) for k in range(eval_iters)]
    hist_n = [sum((h[k] for h in hn), []) for k in range(K_n)]
    t_iter = sum(tp) / n_test        # seconds of batched iteration per team
    rew_p = np.array([[s["reward"] for s in it] for it in hist_p])        # [K][teams]
    rew_n = np.array([[s["reward"] for s in it] for it in hist_n])
    final = rew_p[-1]
    target = final - target_tol * np.abs(final)
    k_p = PR.iterations_to_target(hist_p, target)
    k_n = PR.iterations_to_target(hist_n, target, init_rewards=r_init)
    # first-iteration judge: keep the run whose reward after one iteration is higher
    take_n = rew_n[0] >= rew_p[0]
    k_j = np.where(take_n, k_n, k_p)
    k_j = np.where(k_j == 0, 0, k_j + 1)       # one extra iteration: both starts ran the first one
    final_j = np.where(take_n, rew_n[eval_iters - 1], final)
    reach_p, reach_n, reach_j = k_p <= eval_iters, k_n <= K_n, k_j <= K_n + 1
    both = reach_p & reach_n

    def speed(kp, kn, sel, cap_n):
        tp_ = np.where(reach_p, kp, eval_iters + 1)[sel].mean() * t_iter
        tn_ = np.where(kn <= cap_n, kn, cap_n + 1)[sel].mean() * t_iter + t_infer / n_test
        return float(tp_ / tn_)

    k_p_strict = PR.iterations_to_target(hist_p, final)
    k_n_strict = PR.iterations_to_target(hist_n, final, init_rewards=r_init)
    succ_p = PR.iterations_to_target([[{"reward": float(s["success"])} for s in it] for it in hist_p],
                                     np.ones(n_test))
    succ_n = PR.iterations_to_target([[{"reward": float(s["success"])} for s in it] for it in hist_n],
                                     np.ones(n_test))
    all_t = np.ones(n_test, dtype=bool)
    out = {
        "train_teams": n_train, "test_teams": n_test, "label_samples": label_samples, "label_iterations": label_iters,
        "eval_samples": eval_samples, "eval_iterations": eval_iters, "proposal_iteration_cap": K_n, "epochs": epochs,
        "label_seconds": t_label, "train_seconds": t_train, "final_loss": losses[-1],
        "proposal_used_fraction": float(np.mean(used)),
        "initial_reward_mean": {"zero": 0.0, "proposal": float(r_init.mean())},
        "reward_after_iteration": {"plain": rew_p.mean(1).tolist(), "proposal": rew_n.mean(1).tolist()},
        "success_after_iteration": {"plain": [float(np.mean([s["success"] for s in it])) for it in hist_p],
                                    "proposal": [float(np.mean([s["success"] for s in it])) for it in hist_n]},
        "at_goal_after_iteration": {"plain": [float(np.mean([s["at_goal"] for s in it])) for it in hist_p],
                                    "proposal": [float(np.mean([s["at_goal"] for s in it])) for it in hist_n]},
        "target": f"{100 * (1 - target_tol):.1f} % of the plain planner's reward after {eval_iters} iterations",
        "iterations_to_target_mean": {"plain": float(k_p.mean()),
                                      "proposal_over_reached": float(k_n[reach_n].mean()) if reach_n.any() else None},
        "target_missed_fraction": {"plain": float(1 - reach_p.mean()), "proposal": float(1 - reach_n.mean()),
                                   "proposal_first_iteration_judge": float(1 - reach_j.mean())},
        "time_to_target_speedup": speed(k_p, k_n, all_t, K_n),
        "time_to_target_speedup_both_reached": speed(k_p, k_n, both, K_n) if both.any() else None,
        "time_to_target_speedup_first_iteration_judge": speed(k_p, k_j, all_t, K_n + 1),
        "final_reward_below_plain_fraction": {
            "initial_judge": float((rew_n[eval_iters - 1] < final).mean()),
            "first_iteration_judge": float((final_j < final).mean())},
        "first_iteration_judge_kept_proposal_fraction": float(take_n.mean()),
        "strict_target": {"target_reached_fraction": {"plain": float((k_p_strict <= eval_iters).mean()),
                                                      "proposal": float((k_n_strict <= K_n).mean())}},
        "iterations_to_first_success_mean": {"plain": float(np.minimum(succ_p, eval_iters + 1).mean()),
                                             "proposal": float(np.minimum(succ_n, K_n + 1).mean())},
        "seconds_per_iteration_per_team": t_iter, "proposal_inference_seconds_per_team": t_infer / n_test,
    }
    prop.close()
    return out


SENSITIVITY_DYNAMICS = {
    "diffdrive": W.diffdrive_circle,
    "holo2d": W.holo2d_circle,
    "holo3d": W.holo3d_sphere,
}


def sensitivity(L, dynamics=("diffdrive", "holo2d", "holo3d"), teams=(10, 16), steps=(50, 100, 200, 300),
                iterations=5, runs=30, n_samples=2048, horizon=100, radius=2.0, log=print):
    """Success rate against N and the iteration count (Sec. V-B, Fig. 2).

    One cell is (dynamics, team size, N).  Its runs are the same antipodal
    team (circle in the plane, sphere in space) with independent draws: run j
    is instance j of one batch, so its Philox stream differs from every other
    run's.  A run counts as solved within k iterations when any of its first
    k iterations ends conflict-free (the problem's conditions, Sec. III: the
    controls are feasible by construction); the planner returns the first such
    plan, so the rate cannot fall as k grows.  The rate of plans that also end
    within the goal tolerance is reported beside it."""
    cells = []
    for dyn in dynamics:
        build = SENSITIVITY_DYNAMICS[dyn]
        for n in teams:
            for n_steps in steps:
                p, x0, goal = build(n=n, horizon=horizon, n_samples=n_samples, n_steps=n_steps, radius=radius)
                probs = [p.replace(instance_id=j) for j in range(runs)]
                bc = L.BatchContext(probs, [x0] * runs, [goal] * runs)
                solved = np.zeros(runs, dtype=bool)
                arrived = np.zeros(runs, dtype=bool)
                rate, goal_rate, reward, hits = [], [], [], []
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for k in range(iterations):
                    st = bc.iterate(k)
                    ok = np.array([s["success"] for s in st], dtype=bool)
                    at = np.array([s["at_goal"] for s in st], dtype=bool)
                    solved |= ok
                    arrived |= ok & at
                    rate.append(float(solved.mean()))
                    goal_rate.append(float(arrived.mean()))
                    reward.append(float(np.mean([s["reward"] for s in st])))
                    hits.append(float(np.mean([s["hits"] for s in st])))
                secs = (time.perf_counter() - t0) / iterations
                bc.close()
                cells.append({"dynamics": dyn, "robots": n, "denoising_steps": n_steps,
                              "success_within_iterations": rate, "success_at_goal_within_iterations": goal_rate,
                              "mean_reward_after_iteration": reward, "mean_hits_after_iteration": hits,
                              "seconds_per_iteration_all_runs": secs})
                log(f"{dyn} n={n} N={n_steps}: success within 1..{iterations} iterations "
                    + " ".join(f"{r:.2f}" for r in rate) + f"  ({secs * 1e3:.0f} ms per iteration of {runs} runs)")
    return {"runs_per_cell": runs, "samples": n_samples, "horizon": horizon, "iterations": iterations, "radius": radius,
            "denoising_steps": list(steps), "teams": list(teams), "dynamics": list(dynamics), "cells": cells}


def goal_gap(L, n=16, radius=4.0, n_samples=2048, iterations=20, log=print):
    """Why the plans stop short of their goals (the terminal condition of
    Eqs. problem-conditions, read as every robot within goal_tol at t = T).
    Algorithm 2 from zero controls on the 16-robot antipodal circle (2D
    holonomic, M = 2048), once with the workload's settings and once each with
    a sharper or flatter softmax (lambda), a longer horizon and more
    denoising steps; after every iteration the plan's own trajectory gives each robot's
    final distance to its goal.  Returns per variant the distances (mean,
    median, max over robots) and the conflict-free and at-goal flags by
    iteration."""
    variants = [("workload settings (lambda 0.1, T 100, N 100)", {}),
                ("lambda 0.01", {"temperature": 0.01}),
                ("lambda 0.3", {"temperature": 0.3}),
                ("lambda 1", {"temperature": 1.0}),
                ("lambda 3", {"temperature": 3.0}),
                ("T 150", {"horizon": 150}),
                ("N 300", {"n_steps": 300})]
    out = []
    for label, kw in variants:
        T = kw.get("horizon", 100)
        p, x0, g = W.holo2d_circle(n=n, horizon=T, n_samples=n_samples, radius=radius,
                                   n_steps=kw.get("n_steps", 100))
        if "temperature" in kw:
            p = p.replace(temperature=kw["temperature"])
        x0_d, g_d = L._f32(x0), L._f32(g)
        u = torch.zeros((p.n_robots, p.horizon, p.du), dtype=torch.float32, device="cuda")
        traj = torch.empty((p.n_robots, p.horizon + 1, p.dx), dtype=torch.float32, device="cuda")
        ctx = L.Context(p)
        rows = []
        try:
            for k in range(iterations):
                st = ctx.denoise_iter(x0_d, g_d, u, k, traj=traj)
                d = np.linalg.norm(traj[:, -1, :p.dp].cpu().numpy().astype(np.float64) - g, axis=1)
                rows.append({"iteration": k + 1, "mean_m": float(d.mean()), "median_m": float(np.median(d)),
                             "max_m": float(d.max()), "within_tol": float((d <= p.goal_tol).mean()),
                             "success": bool(st["success"]), "at_goal": bool(st["at_goal"]),
                             "reward": float(st["reward"])})
        finally:
            ctx.close()
        # one more iteration from the final plan through the split calls, not
        # applied: the softmax weights' effective sample count (sum w)^2 /
        # sum w^2 at the first, middle and last denoising steps, and the size
        # of the deformation the iteration would add
        du = torch.zeros(p.D, dtype=torch.float32, device="cuda")
        ub = u.reshape(-1).contiguous()
        ess = {}
        for i in range(p.n_steps, 0, -1):
            eps, r, _ = L.sample_rollout_fitness(p, x0_d, g_d, ub, du, iterations, i)
            du, w = L.score_update(p, r, eps, du, i)
            if i in (p.n_steps, p.n_steps // 2, 1):
                w64 = w.double()
                ess[i] = float(w64.sum() ** 2 / (w64 * w64).sum())
        dU_rms = float(du.double().pow(2).mean().sqrt())
        last = rows[-1]
        log(f"{label}: after {iterations} iterations final distance mean {last['mean_m']:.3f} m, "
            f"max {last['max_m']:.3f} m, robots within {p.goal_tol} m {last['within_tol']:.2f}, "
            f"conflict-free {last['success']}")
        log(f"  next iteration: effective samples {', '.join(f'step {i}: {v:.1f}' for i, v in ess.items())}; "
            f"deformation rms {dU_rms:.3f}")
        out.append({"variant": label, "goal_tol": p.goal_tol, "by_iteration": rows,
                    "next_iteration_effective_samples": {str(i): v for i, v in ess.items()},
                    "next_iteration_deformation_rms": dU_rms})
    return out


def first_success(L, scenario="circle", n=16, runs=50, n_samples=2048, horizon=100, n_steps=100, radius=4.0,
                  deadline_s=5.0, max_iterations=500, seed=0, temperature=None, log=print):
    """Wall time to the first conflict-free plan (Sec. V-C, the paper's
    headline measure), single-problem path, 2D holonomic robots.

    scenario "circle": n robots on an antipodal circle of the given radius,
    run j drawing from its own Philox stream (instance id j).  "random":
    start and goal sets drawn uniformly, at least 1 m apart, in a square whose
    side is the circle's diameter (Sec. V-D), one instance per run.  The
    clock covers the whole planning call, context set-up included, and stops
    when an iteration returns a conflict-free plan or at the deadline.
    temperature replaces the workload's softmax temperature lambda (0.1) when
    given: the reading of the batch normalisation that Sec. IV-C leaves open
    sets how flat the weights are."""
    import math
    rng = np.random.default_rng(seed)
    p0, x00, g0 = W.holo2d_circle(n=n, horizon=horizon, n_samples=n_samples, n_steps=n_steps, radius=radius)
    if temperature is not None:
        p0 = p0.replace(temperature=float(temperature))
    # untimed warm-up: library load, first graph capture
    L.plan(p0, x00, g0, iterations=1)
    torch.cuda.synchronize()
    times, iters, solved = [], [], []
    for j in range(runs):
        if scenario == "circle":
            p, x0, g = p0.replace(instance_id=j), x00, g0
        else:
            p, x0, g = W.random_instance(rng, W.HOLO2D, n, horizon, n_samples, box=2.0 * radius, min_sep=1.0,
                                         n_steps=n_steps)
            p = p.replace(instance_id=j, temperature=p0.temperature)
        t0 = time.perf_counter()
        x0_d, g_d = L._f32(x0), L._f32(g)
        u = torch.zeros((p.n_robots, p.horizon, p.du), dtype=torch.float32, device="cuda")
        ctx = L.Context(p)
        ok, k = False, 0
        try:
            while k < max_iterations and time.perf_counter() - t0 < deadline_s:
                st = ctx.denoise_iter(x0_d, g_d, u, k)
                k += 1
                if st["success"]:
                    ok = True
                    break
        finally:
            ctx.close()
        dt = time.perf_counter() - t0
        solved.append(ok)
        iters.append(k)
        if ok:
            times.append(dt)
    solved = np.array(solved)
    t = np.array(times) if times else np.array([math.nan])
    log(f"{scenario} n={n}: solved {solved.mean():.2f} within {deadline_s} s, mean time to first success "
        f"{t.mean() * 1e3:.1f} ms (median {np.median(t) * 1e3:.1f} ms), mean iterations {np.mean(iters):.2f}")
    return {"scenario": scenario, "robots": n, "runs": runs, "samples": n_samples, "horizon": horizon,
            "denoising_steps": n_steps, "radius_or_half_side": radius, "deadline_s": deadline_s,
            "temperature": float(p0.temperature),
            "solved_fraction": float(solved.mean()), "mean_seconds_to_first_success": float(t.mean()),
            "median_seconds_to_first_success": float(np.median(t)),
            "mean_iterations": float(np.mean(iters)),
            "iterations_of_solved_runs": [int(i) for i, s in zip(iters, solved) if s]}


def gemm_roofline(L, rows=640, width=256, hidden=512, d_out=200, batch=64, large=8192, reps=50, log=print):
    """Achieved throughput of the proposal's BF16 MFMA product kernel
    (d4p_gemm_bf16) at the shapes one training step runs (rows = robots of a
    64-team batch) and at a large square shape, against the 2.5 PFLOP/s dense
    BF16 peak.  Each shape is launched `reps` times back to back between HIP
    events on the launch stream; flops = 2 M N K per launch."""
    peak = 2.5e15
    shapes = [
        ("layer in, forward: [R x W] [W x H]", rows, hidden, width, False, False),
        ("layer out, forward: [R x H] [H x W]", rows, width, hidden, False, False),
        ("pool: [B x W] [W x W]", batch, width, width, False, False),
        ("head: [R x W] [W x T d_u]", rows, d_out, width, False, False),
        ("weight gradient: [R x W]^T [R x H]", width, hidden, rows, True, False),
        ("input gradient: [R x H] [W x H]^T", rows, width, hidden, False, True),
        (f"large square {large}", large, large, large, False, False),
        (f"large square {large}, B transposed", large, large, large, False, True),
    ]
    out = []
    s = torch.cuda.current_stream()
    for name, M, N, K, ta, tb in shapes:
        A = (torch.randn((K, M) if ta else (M, K), device="cuda") * 0.1).to(torch.bfloat16)
        B = (torch.randn((N, K) if tb else (K, N), device="cuda") * 0.1).to(torch.bfloat16)
        C = torch.zeros((M, N), device="cuda")
        n_rep = reps if M * N * K < 1e11 else 5
        for _ in range(3):
            L.gemm_bf16(A, B, M, N, K, ta, tb, C=C)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(n_rep):
            L.gemm_bf16(A, B, M, N, K, ta, tb, C=C)
        e1.record(s)
        e1.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / n_rep
        # spot check against a float32 product of the same BF16 operands
        ref = (A.float().t() if ta else A.float()) @ (B.float().t() if tb else B.float())
        err = float((C - ref).abs().max() / ref.abs().max().clamp_min(1e-30))
        flops = 2.0 * M * N * K
        row = {"shape": name, "M": M, "N": N, "K": K, "us": t * 1e6, "tflops": flops / t / 1e12,
               "frac_of_peak": flops / t / peak, "max_rel_err": err}
        log(f"{name}: {t * 1e6:.2f} us, {flops / t / 1e12:.2f} TFLOP/s ({flops / t / peak:.4f} of peak)")
        out.append(row)
    return out
