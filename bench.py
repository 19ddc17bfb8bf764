"""Benchmark of the denoising hot path on one MI355X.

A step is one deformation iteration (Algorithm 2 loop body): N = 100
denoising steps of Algorithm 1 (sampling, rollout, reward, softmax weights,
weighted update) plus the final apply-and-rollout, on the 16-robot 3D
holonomic sphere swap with T = 100 and M = 8192 samples.  The metric is
robot*step*samples per second: n * T * M * N per iteration over the measured
wall time of the iteration, inputs resident in device memory.

The JSON line also carries:
  roofline      the fused sample+rollout+reward kernel (the dominant kernel):
                algorithmic VALU operations per launch (the method's work per
                robot*step*sample, pair checks of every pair at every step
                included) over its average launch time, measured with HIP
                events on its stream, against the chip's FP32 vector peak of
                78.6 T lane-operations/s (157.3 TFLOP/s counting an FMA as
                two); the peak of the kernel's own instruction mix is a
                secondary figure.
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload,
                on every host core this process may use (at most 16).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# gfx950 VALU issue classes (256 CUs x 4 SIMDs at 2.4 GHz), lanes per second.
# The 157.3 TFLOP/s FP32 vector figure is 32 lanes per SIMD and cycle: a
# wave64 instruction in 2 cycles.  That full rate holds for FP32 add,
# subtract, multiply and fused multiply-add, and for 32-bit integer add,
# subtract, logic (three-input bitop3 included), shifts and moves, when every
# operand is a VGPR, an inline constant or a literal.  Compares, selects,
# min/max/median, conversions, 32-bit multiplies and the 32x32->64 product,
# three-operand integer forms (add3, shift-add, and-or), bit-field extracts
# and any instruction with a scalar-register operand issue at half that rate
# (4 cycles); transcendentals (reciprocal, square root, exp, sin) at a quarter
# (8 cycles).  A throughput probe of 16 independent chains per lane, one
# instruction form at a time, measures 2.3-2.9, 4.1-4.8 and 8.1-8.5 cycles.
SIMD_HZ = 256 * 4 * 2.4e9
FULL_RATE = SIMD_HZ * 32
HALF_RATE = SIMD_HZ * 16
QUARTER_RATE = SIMD_HZ * 8
HBM_PEAK_GBS = 8000.0

# Algorithmic VALU operations per robot*step*sample of the fused kernel: the
# operations each step of the method needs in its leanest gfx950 form (one
# VALU instruction per arithmetic step, a fused multiply-add, a clamp as one
# median, a 32x32->64 product counted once), independent of how the kernel
# schedules them, split into the (full, half, quarter) rate classes above:
#  - standard normal, per block of 4: Philox4x32-10 = 10 rounds of two
#    32x32->64 products (half) and two three-input XORs (full), and 2 full for
#    the counter; per Box-Muller pair: uniform 3 full + 1 half (conversion);
#    ln: range reduction 4 full + 5 half, division 8 full + 1 reciprocal,
#    series and e*ln2 9 full; -2 ln 1 full; corrected square root 4 full +
#    4 half + 1 square root; sin/cos with the quarter-turn rotation 22 full +
#    4 half; two products 2 full.  Per normal: 32 full + 12 half + 1 quarter.
#  - sampled control: two fused multiply-adds and a clamp per component
#  - dynamics per step: double integrator 3 full + 1 half (speed clamp) per
#    axis; unicycle 11 full + 4 quarter (two heading updates, the mid-step and
#    end-of-step sin/cos with their range scaling, Simpson sums); differential
#    drive 17 full + 1 half + 4 quarter (the speed's two steps, its clamp)
#  - goal term: differences, squared distance, square root, fused step, sum:
#    2 d_p + 2 full + 1 quarter
#  - bounding box of the block: running min and max, 2 d_p half
#  - broad phase: (n - 1)/2 partners per robot and block of Tb steps; per
#    partner the box gap (2 differences full and a three-way max half per
#    axis), squares and sums d_p full, compare half, or full:
#    3 d_p + 1 full + d_p + 1 half
#  - collision flags: 3 full
#  - static obstacles: per obstacle and step, differences, squared distance,
#    or full and the compare half: 2 d_p + 1 full + 1 half
# The exact pair checks of partners the broad phase keeps are data dependent
# and not counted.
NORMAL_OPS = (32.0, 12.0, 1.0)


def ops_per_unit(dyn, n, steps_per_block, n_obstacles=0):
    """Algorithmic (full, half, quarter rate) VALU operations per robot*step*sample."""
    from paper_2503_12204_amd import workloads as W
    dx, du, dp = W.dims(dyn)
    dyn_ops = {W.UNICYCLE: (11, 0, 4), W.DIFFDRIVE: (17, 1, 4)}.get(dyn, (3 * dp, dp, 0))
    pairs = (n - 1) / 2.0 / steps_per_block
    full = du * NORMAL_OPS[0] + 2 * du + dyn_ops[0] + (2 * dp + 2) + pairs * (3 * dp + 1) + 3
    half = du * NORMAL_OPS[1] + du + dyn_ops[1] + 2 * dp + pairs * (dp + 1)
    quarter = du * NORMAL_OPS[2] + dyn_ops[2] + 1
    full += n_obstacles * (2 * dp + 1)
    half += n_obstacles * 1
    return full, half, quarter


# The method's work per robot*step*sample in VALU lane-operations, the
# roofline's numerator: d_u normal draws at 40 operations each (Philox and
# Box-Muller), 3 d_u to form and clip the sampled control, the dynamics (a
# double integrator's exact step 5 per axis, a unicycle or differential drive
# RK4 step about 80 with its sines and cosines), 8 for the goal term, and the
# pair term of Eq. generic-reward: (n - 1)/2 pair checks per robot and step at
# 2 d_p + 2 each (differences, squares and sums, compare, flag); a static
# obstacle costs one such check per robot and step.  This is what the method
# computes, whatever the kernel skips: the exact broad phase of the kernel
# avoids most pair checks and earns that as speed.  At 16 robots in 3D:
# 120 + 9 + 15 + 8 + 60 = 212.
def algorithmic_ops(dyn, n, n_obstacles=0):
    from paper_2503_12204_amd import experiments as E
    return E.algorithmic_ops(dyn, n, n_obstacles)


def issue_seconds_per_unit(ops):
    """Ideal VALU time of one robot*step*sample at the issue rates above."""
    full, half, quarter = ops
    return full / FULL_RATE + half / HALF_RATE + quarter / QUARTER_RATE


WORKLOADS = {
    "holo3d_sphere_swap": "16 robots, 3D holonomic double integrator, antipodal sphere swap, T=100, M=8192, N=100",
    "unicycle_random": "8 unicycles, random starts/goals in a 10 m box, T=100, M=2048, N=100",
    "holo2d_circle_swap": "4 robots, 2D holonomic double integrator, antipodal circle swap, T=50, M=256, N=100",
    "diffdrive_circle_swap": "16 robots, differential drive (x = [p, theta, v], u = [omega, a]), antipodal circle "
                             "swap, T=100, M=8192, N=100",
    "holo2d_circle_obstacles": "16 robots, 2D holonomic double integrator, antipodal circle swap around 4 static "
                               "discs, T=100, M=8192, N=100",
}


def make_workload(name):
    from paper_2503_12204_amd import workloads as W
    if name == "holo3d_sphere_swap":
        return W.holo3d_sphere()
    if name == "unicycle_random":
        return W.unicycle_random()
    if name == "holo2d_circle_swap":
        return W.holo2d_circle()
    if name == "diffdrive_circle_swap":
        return W.diffdrive_circle(n=16, horizon=100, n_samples=8192)
    if name == "holo2d_circle_obstacles":
        return W.holo2d_circle_obstacles(n=16, n_obs=4, horizon=100, n_samples=8192)
    raise SystemExit(f"unknown workload {name}")


def _oracle_shard(job):
    """One CPU worker of cpu_baseline: the oracle, untouched and single-
    threaded, on samples [lo, hi) of consecutive denoising steps for about
    target_s seconds.  Returns (robot*step*samples, seconds, steps)."""
    name, lo, hi, target_s = job
    from threadpoolctl import threadpool_limits
    from oracle import mbd as ombd
    from oracle import schedule as osched
    p, x0, g = make_workload(name)
    sched = osched.step_scalars(p.n_steps, p.beta_min, p.beta_max)
    ms, sg, os_ = sched
    du = np.zeros(p.D)
    ub = np.zeros(p.D)
    steps = 0
    i = p.n_steps
    with threadpool_limits(limits=1):  # one core, whatever BLAS the oracle's NumPy would use
        t0 = time.perf_counter()
        while True:
            out = ombd.sample_rewards(p, x0, g, ub, du, 0, i, sched=sched, samples=np.arange(lo, hi))
            du, _ = ombd.mc_update(du, out["eps"], out["r"], ms[i], sg[i], os_[i], p.temperature, True)
            steps += 1
            i -= 1
            if time.perf_counter() - t0 >= target_s or i == 0:
                break
        dt = time.perf_counter() - t0
    return p.n_robots * p.horizon * (hi - lo) * steps, dt, steps


def cpu_baseline(name, target_s=10.0, workers=None):
    """The oracle, untouched, on a bounded sample of the workload, on every
    host core this process may use (at most 16): worker w runs sampling,
    rollout, reward and the weighted update of consecutive denoising steps on
    its own slice of the first min(M, 1024 W) samples, single-threaded, for
    about target_s seconds; the rate is the workers' total work over the
    longest worker's time.  The workers are forked processes that run only
    NumPy (no GPU call)."""
    import multiprocessing as mp
    p, _, _ = make_workload(name)
    W = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    total = min(p.n_samples, 1024 * W)
    W = min(W, total)
    edges = [total * w // W for w in range(W + 1)]
    jobs = [(name, edges[w], edges[w + 1], target_s) for w in range(W)]
    try:
        with mp.get_context("fork").Pool(W) as pool:
            res = pool.map(_oracle_shard, jobs)
    except Exception as exc:  # no worker processes here: one in-process worker
        print(f"cpu_baseline: worker processes failed ({exc}); timing one core", file=sys.stderr, flush=True)
        W, total = 1, min(p.n_samples, 1024)
        res = [_oracle_shard((name, 0, total, target_s))]
    units = sum(r[0] for r in res)
    dt = max(r[1] for r in res)
    steps = min(r[2] for r in res)
    return {"value": units / dt, "unit": "robot*step*samples/s", "cores": W, "kind": "oracle",
            "sample": f"{steps}+ denoising steps of {name} on samples 0..{total - 1}, split over {W} "
                      f"single-threaded worker processes (sampling, FP64 rollout, reward, weighted update), "
                      f"{dt:.1f} s"}


# the kernels and the host rule that picks their launch shape
KERNEL_SOURCES = ["paper_2503_12204_amd/csrc/d4_device.hpp", "paper_2503_12204_amd/csrc/d4_kernels.hpp",
                  "paper_2503_12204_amd/csrc/d4_api.hip", "paper_2503_12204_amd/csrc/d4_host.hpp"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload):
    """HBM bytes per launch of the fused kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by a copy calibration),
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"k_rollfit_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("    ") and ":" in line:
                k, v = line.strip().split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != kernel_source_hash():
        return None
    return float(vals["traffic_bytes_per_launch"])


def time_fused_kernel(L, p, x0, g, reps=30):
    """Average duration of the fused sample+rollout+reward kernel on the zero
    plan, bracketed by HIP events on the stream it is launched on (torch's
    current stream).  Used for the counter runs."""
    import torch
    D, M = p.D, p.n_samples
    eps = torch.empty((D, M), dtype=torch.float32, device="cuda")
    r = torch.empty(M, dtype=torch.float32, device="cuda")
    hits = torch.empty(M, dtype=torch.int32, device="cuda")
    ub = torch.zeros(D, dtype=torch.float32, device="cuda")
    du = torch.zeros(D, dtype=torch.float32, device="cuda")
    for _ in range(3):
        L.sample_rollout_fitness(p, x0, g, ub, du, 0, p.n_steps, eps, r, hits)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for k in range(reps):
        L.sample_rollout_fitness(p, x0, g, ub, du, 0, p.n_steps - (k % p.n_steps), eps, r, hits)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def time_fused_kernel_in_iteration(L, p, x0, g, u, iteration):
    """Average duration of the fused kernel over the N denoising steps of one
    iteration from plan u.  The iteration runs first through the split calls
    (the launches of d4_denoise_iter), keeping each step's Delta U_i; the N
    fused launches are then replayed back to back on those inputs between
    two HIP events on the launch stream."""
    import torch
    D, M = p.D, p.n_samples
    eps = torch.empty((D, M), dtype=torch.float32, device="cuda")
    r = torch.empty(M, dtype=torch.float32, device="cuda")
    hits = torch.empty(M, dtype=torch.int32, device="cuda")
    ub = u.reshape(-1).contiguous()
    w = torch.empty(M, dtype=torch.float32, device="cuda")
    dus = [torch.zeros(D, dtype=torch.float32, device="cuda")]
    steps = list(range(p.n_steps, 0, -1))
    for i in steps:
        L.sample_rollout_fitness(p, x0, g, ub, dus[-1], iteration, i, eps, r, hits)
        dus.append(L.score_update(p, r, eps, dus[-1], i, None, w)[0])
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for k, i in enumerate(steps):
        L.sample_rollout_fitness(p, x0, g, ub, dus[k], iteration, i, eps, r, hits)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / len(steps) * 1e-3


def time_update_kernel(L, p, x0, g, u, iteration, reps=20):
    """Average duration of the update kernel (statistics, softmax, weighted
    row reduction) on one step's draws and rewards, launched back to back
    between HIP events on the launch stream."""
    import torch
    D, M = p.D, p.n_samples
    eps = torch.empty((D, M), dtype=torch.float32, device="cuda")
    r = torch.empty(M, dtype=torch.float32, device="cuda")
    hits = torch.empty(M, dtype=torch.int32, device="cuda")
    du = torch.zeros(D, dtype=torch.float32, device="cuda")
    du_out = torch.empty(D, dtype=torch.float32, device="cuda")
    w = torch.empty(M, dtype=torch.float32, device="cuda")
    L.sample_rollout_fitness(p, x0, g, u.reshape(-1).contiguous(), du, iteration, p.n_steps, eps, r, hits)
    L.score_update(p, r, eps, du, p.n_steps, du_out, w)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        L.score_update(p, r, eps, du, p.n_steps, du_out, w)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def time_update_kernel_cold(L, p, x0, g, u, iteration, reps=6):
    """Median duration of single update launches, each after 1 GiB of other
    data has been read through the caches (HBM reads, no Infinity Cache hits
    on the draws)."""
    import torch
    D, M = p.D, p.n_samples
    eps = torch.empty((D, M), dtype=torch.float32, device="cuda")
    r = torch.empty(M, dtype=torch.float32, device="cuda")
    hits = torch.empty(M, dtype=torch.int32, device="cuda")
    du = torch.zeros(D, dtype=torch.float32, device="cuda")
    du_out = torch.empty(D, dtype=torch.float32, device="cuda")
    w = torch.empty(M, dtype=torch.float32, device="cuda")
    flush = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    L.sample_rollout_fitness(p, x0, g, u.reshape(-1).contiguous(), du, iteration, p.n_steps, eps, r, hits)
    s = torch.cuda.current_stream()
    times = []
    for k in range(reps):
        # read 1 GiB of other data (reads leave no dirty lines to write back)
        flush.sum()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        L.score_update(p, r, eps, du, p.n_steps, du_out, w)
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    del flush
    return float(np.median(times))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="holo3d_sphere_swap", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="choose the workload's tile with d4_autotune (whole iterations) before timing")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--kernel-only", type=int, default=0,
                    help="only launch the fused kernel this many times (for counter runs)")
    ap.add_argument("--source-hash", action="store_true", help="print the kernel source hash and exit")
    ap.add_argument("--experiment", choices=["batched", "proposal", "sensitivity", "first_success", "gemm", "goal_gap"],
                    default=None,
                    help="time-to-target of the batched or learned-proposal form against the plain planner, "
                         "or the success-rate sweep over denoising steps and iterations")
    ap.add_argument("--runs", type=int, default=30, help="runs per cell of the sensitivity sweep")
    ap.add_argument("--success-runs", type=int, default=50, help="runs per scenario of first_success")
    ap.add_argument("--scenarios", default="circle,random", help="scenarios of first_success")
    ap.add_argument("--temperature", type=float, default=None,
                    help="softmax temperature of first_success (default: the workload's 0.1)")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched experiment: time the batched form only (for profiling runs)")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched experiment: keep the rule's tiles (no bucket autotuning)")
    ap.add_argument("--radius", type=float, default=None,
                    help="circle (sphere) radius, m: 2 for the sensitivity sweep, 4 for first_success by default")
    ap.add_argument("--dynamics", default="diffdrive,holo2d,holo3d", help="dynamics of the sensitivity sweep")
    ap.add_argument("--teams", default="10,16", help="team sizes of the sensitivity sweep")
    ap.add_argument("--train-teams", type=int, default=4096)
    ap.add_argument("--test-teams", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=20)
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the planner's hot path runs on a single device "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.experiment and not args.kernel_only and not args.no_cpu_baseline:
        # the oracle's worker processes are forked before this process
        # touches the GPU (torch and the HIP library are not loaded yet)
        cpu = cpu_baseline(args.workload, args.cpu_seconds)

    import torch
    from paper_2503_12204_amd import _lib as L
    from paper_2503_12204_amd import workloads as W

    torch.cuda.set_device(0)
    if args.experiment:
        from paper_2503_12204_amd import experiments as E

        def log(msg):
            print(msg, file=sys.stderr, flush=True)

        if args.experiment == "batched":
            res = E.batched_vs_plain(L, plain=not args.no_plain, tune=not args.no_tune, log=log)
            out = {"metric": "time-to-target speedup of the batched form over the plain planner",
                   "value": res.get("speedup"), "unit": "x", "n_gpus": 1, "higher_is_better": True,
                   "dtype": "f32", "data": "synthetic",
                   "config": {"workload": "batched_mix", "description": "512 instances, robots U{2..32}, "
                              "horizon U{40..160}, 3 dynamics, M=1024, N=100, random starts/goals in a 10 m box"},
                   "details": res}
        elif args.experiment == "gemm":
            res = E.gemm_roofline(L, log=log)
            head = res[0]
            out = {"metric": "BF16 MFMA product throughput of the proposal network (training-step shapes)",
                   "value": head["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "higher_is_better": True,
                   "dtype": "bf16 in, f32 accumulate", "data": "synthetic",
                   "config": {"workload": "proposal_gemm", "description": "d4p_gemm_bf16 at the shapes of one "
                              "training step (64 teams, about 640 robots, width 256, hidden 512, T d_u = 200) and "
                              "one large square product"},
                   "roofline": {"bound": "mfma", "achieved": head["tflops"], "peak": 2500.0, "unit": "TFLOP/s",
                                "frac": head["frac_of_peak"], "traffic": None},
                   "details": res}
        elif args.experiment == "first_success":
            res = [E.first_success(L, scenario=sc, n=t, radius=args.radius or 4.0, runs=args.success_runs,
                                   temperature=args.temperature, log=log)
                   for sc in args.scenarios.split(",") for t in (int(x) for x in args.teams.split(","))]
            head = [r for r in res if r["scenario"] == "circle" and r["robots"] == 16] or res
            out = {"metric": "mean wall time to the first conflict-free plan, 16 robots 2D holonomic, antipodal circle",
                   "value": head[0]["mean_seconds_to_first_success"], "unit": "s", "n_gpus": 1,
                   "higher_is_better": False, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": "first_success", "description": "2D holonomic teams, antipodal circle of "
                              f"radius {args.radius or 4.0} m and random targets in a square of the circle's diameter, "
                              f"T=100, M=2048, N=100, 5 s deadline, {args.success_runs} runs each"},
                   "details": res}
        elif args.experiment == "goal_gap":
            res = E.goal_gap(L, radius=args.radius or 4.0, log=log)
            out = {"metric": "mean final distance to goal after 20 iterations, 16 robots 2D holonomic, antipodal circle",
                   "value": res[0]["by_iteration"][-1]["mean_m"], "unit": "m", "n_gpus": 1,
                   "higher_is_better": False, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": "goal_gap", "description": f"antipodal circle of radius {args.radius or 4.0} m, "
                              "T=100, M=2048, N=100, and variants of lambda, T and N"},
                   "details": res}
        elif args.experiment == "sensitivity":
            res = E.sensitivity(L, dynamics=tuple(args.dynamics.split(",")),
                                teams=tuple(int(t) for t in args.teams.split(",")), runs=args.runs,
                                radius=args.radius or 2.0, log=log)
            mid = [c for c in res["cells"] if c["denoising_steps"] == 100]
            out = {"metric": "success rate within the iteration budget, mean over dynamics and team sizes at N=100",
                   "value": float(np.mean([c["success_within_iterations"][-1] for c in mid])), "unit": "fraction",
                   "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": "sensitivity", "description": f"antipodal circle (sphere in 3D) of radius "
                              f"{args.radius or 2.0} m, teams of {args.teams} robots, dynamics {args.dynamics}, T=100, M=2048, "
                              "N in {50, 100, 200, 300}, 5 iterations, independent runs per cell"},
                   "details": res}
        else:
            res = E.proposal_gain(L, n_train=args.train_teams, n_test=args.test_teams, epochs=args.epochs, log=log)
            out = {"metric": "time-to-target speedup of the learned proposal over the plain planner",
                   "value": res["time_to_target_speedup"], "unit": "x", "n_gpus": 1, "higher_is_better": True,
                   "dtype": "f32 planner, bf16 network", "data": "synthetic",
                   "config": {"workload": "learned_proposal", "description": "2D holonomic teams of 4..16 robots, "
                              "random starts/goals in a 10 m box, T=100, N=100, evaluation at M=2048"},
                   "details": res}
        print(json.dumps(out), flush=True)
        return
    p, x0n, gn = make_workload(args.workload)
    x0 = torch.as_tensor(x0n, device="cuda")
    g = torch.as_tensor(gn, device="cuda")

    if args.kernel_only:
        print(f"fused kernel and update kernel x{args.kernel_only} on {args.workload}", flush=True)
        time_fused_kernel(L, p, x0, g, reps=args.kernel_only)
        D, M = p.D, p.n_samples
        eps = torch.empty((D, M), dtype=torch.float32, device="cuda")
        r = torch.empty(M, dtype=torch.float32, device="cuda")
        hits = torch.empty(M, dtype=torch.int32, device="cuda")
        zero = torch.zeros(D, dtype=torch.float32, device="cuda")
        L.sample_rollout_fitness(p, x0, g, zero, zero, 0, p.n_steps, eps, r, hits)
        du_out = torch.empty(D, dtype=torch.float32, device="cuda")
        for _ in range(args.kernel_only):
            L.score_update(p, r, eps, zero, p.n_steps, du_out, None)
        n_bytes = 256 << 20
        a = torch.empty(n_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print("copy calibration: 256 MiB read + 256 MiB write", flush=True)
        return

    if args.tune:
        from paper_2503_12204_amd import autotune as AT
        AT.tune(p, x0n, gn, force=True)
    u = torch.zeros((p.n_robots, p.horizon, p.du), dtype=torch.float32, device="cuda")
    ctx = L.Context(p)
    for k in range(args.warmup):
        ctx.denoise_iter(x0, g, u, k, sync=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ctx.denoise_iter(x0, g, u, args.warmup + k, sync=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = ctx.denoise_iter(x0, g, u, args.warmup + args.steps)
    ctx.close()
    ms_per_step = elapsed / args.steps * 1e3
    units = p.n_robots * p.horizon * p.n_samples * p.n_steps
    value = units / (elapsed / args.steps)

    t_k = time_fused_kernel_in_iteration(L, p, x0, g, u, args.warmup + args.steps + 1)
    from paper_2503_12204_amd import autotune as AT
    S_t, Tb_t, R_t = AT.get_tile(p)
    units = p.n_robots * p.horizon * p.n_samples
    opu = algorithmic_ops(p.dyn, p.n_robots, len(p.obstacles))
    achieved = opu * units / t_k
    # secondary: the kernel's own operation mix against its ideal issue time
    opc = ops_per_unit(p.dyn, p.n_robots, Tb_t, len(p.obstacles))
    mix_peak = sum(opc) / issue_seconds_per_unit(opc)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": FULL_RATE / 1e12,
                "unit": "T lane-ops/s", "frac": achieved / FULL_RATE, "traffic": stored_traffic(args.workload),
                "kernel": "k_rollfit (fused sample+rollout+reward)", "kernel_us": t_k * 1e6,
                "ops_per_unit": opu, "units_per_launch": units,
                "tile": {"samples_per_group": S_t, "steps_per_block": Tb_t, "replicas": R_t},
                "issue_mix": {"ops_per_unit_full_half_quarter": list(opc),
                              "achieved": sum(opc) * units / t_k / 1e12, "peak": mix_peak / 1e12,
                              "frac": sum(opc) * units / t_k / mix_peak}}
    # the weighted reduction: HBM-bound; algorithmic bytes = the draws read
    # once, the rewards, Delta U in and out, and the weights written once.
    # In the iteration the draws come straight from the fused kernel and part
    # of them from the 256 MB Infinity Cache; the cold figure first reads
    # 1 GiB of other data through the caches before each timed launch.
    t_u = time_update_kernel(L, p, x0, g, u, args.warmup + args.steps + 2)
    t_uc = time_update_kernel_cold(L, p, x0, g, u, args.warmup + args.steps + 2)
    upd_bytes = 4 * (p.D * p.n_samples + 2 * p.n_samples + 2 * p.D)
    update = {"bound": "hbm", "achieved": upd_bytes / t_u / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": upd_bytes / t_u / 1e9 / HBM_PEAK_GBS, "kernel": "k_softmax_update (statistics, softmax, "
              "weighted row reduction, update)", "kernel_us": t_u * 1e6, "bytes_per_launch": upd_bytes,
              "cold": {"kernel_us": t_uc * 1e6, "achieved": upd_bytes / t_uc / 1e9,
                       "frac": upd_bytes / t_uc / 1e9 / HBM_PEAK_GBS}}
    out = {
        "metric": "robot*step*samples/s in rollout+fitness (whole denoising iteration)",
        "value": value, "unit": "robot*step*samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "robots": p.n_robots, "horizon": p.horizon, "samples": p.n_samples,
                   "denoising_steps": p.n_steps, "dynamics": W.DYN_NAMES[p.dyn]},
        "roofline": roofline,
        "update_kernel_roofline": update,
        "last_iteration": {"reward": st["reward"], "hits": st["hits"], "success": st["success"],
                           "at_goal": st["at_goal"]},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
