"""Batched form: uneven instances advanced together must reproduce each
instance's single-problem iteration bit for bit, and their final rewards must
match the oracle's reward of the same plans."""
import numpy as np
import pytest
import torch

from oracle import mbd as ombd
from paper_2503_12204_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "the GPU tests need a HIP device"
    from paper_2503_12204_amd import _lib
    return _lib


def _mix(count, M, N, seed=0, n_range=(2, 32), t_range=(9, 61)):
    out = W.batched_mix(count=count, n_samples=M, n_range=n_range, t_range=t_range, seed=seed)
    return [(p.replace(n_steps=N), x0, g) for p, x0, g in out]


def test_batch_equals_single_problem_runs(L):
    # M = 160: the single-problem path updates with its one-wave form
    # (k_softmax_update_wave), the batched form with four waves per
    # workgroup; both must give the same plans bit for bit
    inst = _mix(7, 160, 12, seed=3)
    inst.append(W.holo3d_sphere(n=32, horizon=20, n_samples=160))
    inst[-1] = (inst[-1][0].replace(n_steps=12, instance_id=7), inst[-1][1], inst[-1][2])
    # obstacles are per instance (appendix penalty); the paper's differential drive too
    q, x0q, gq = W.holo2d_circle_obstacles(n=6, n_obs=2, horizon=20, n_samples=160)
    inst.append((q.replace(n_steps=12, instance_id=8), x0q, gq))
    q, x0q, gq = W.diffdrive_circle(n=5, horizon=22, n_samples=160)
    inst.append((q.replace(n_steps=12, instance_id=9), x0q, gq))
    probs = [p for p, _, _ in inst]
    print("shapes", [(p.dyn, p.n_robots, p.horizon) for p in probs], flush=True)
    bc = L.BatchContext(probs, [x for _, x, _ in inst], [g for _, _, g in inst])
    rng = np.random.default_rng(1)
    plans = [rng.uniform(-0.5, 0.5, size=(p.n_robots, p.horizon, p.du)).astype(np.float32) for p in probs]
    bc.set_plans(plans)
    for it in range(2):
        stats = bc.iterate(it)
    got = [bc.plan_of(j).cpu().numpy() for j in range(len(probs))]
    bc.close()
    from paper_2503_12204_amd import autotune as AT
    for j, (p, x0, g) in enumerate(inst):
        # the single-problem path with the batched form's tile
        S, Tb, R = AT.get_tile(p, batched=True)
        AT.set_tile(p.dyn, p.n_robots, p.horizon, S, Tb, R)
        try:
            ctx = L.Context(p)
            u = torch.as_tensor(plans[j], device="cuda").clone()
            for it in range(2):
                st = ctx.denoise_iter(torch.as_tensor(x0, device="cuda"), torch.as_tensor(g, device="cuda"), u, it)
            ctx.close()
        finally:
            AT.clear_tile(p.dyn, p.n_robots, p.horizon)
        assert np.array_equal(u.cpu().numpy(), got[j]), f"instance {j}"
        assert st == stats[j], f"instance {j}"
        fin = ombd.apply_deformation(p, x0, g, got[j], np.zeros(p.D))
        assert abs(stats[j]["reward"] - fin["r"]) <= 1e-3 * abs(fin["r"])
        assert stats[j]["hits"] == fin["hits"]


def test_batch_rejects_mixed_sampler_settings(L):
    inst = _mix(2, 64, 5)
    probs = [inst[0][0], inst[1][0].replace(temperature=0.2)]
    with pytest.raises(L.D4Error):
        L.BatchContext(probs, [x for _, x, _ in inst], [g for _, _, g in inst])


def test_sensitivity_sweep_cells(L):
    """The success-rate sweep (Sec. V-B) on a tiny grid: one cell per
    (dynamics, team, N), rates that never fall with more iterations, and
    independent draws per run."""
    from paper_2503_12204_amd import experiments as E
    print("sensitivity sweep: 3 dynamics x n=4 x N in {6, 12}, 3 runs, M=128, T=16", flush=True)
    res = E.sensitivity(L, teams=(4,), steps=(6, 12), iterations=3, runs=3, n_samples=128, horizon=16,
                        log=lambda m: print(m, flush=True))
    cells = res["cells"]
    assert [(c["dynamics"], c["denoising_steps"]) for c in cells] == [
        (d, N) for d in ("diffdrive", "holo2d", "holo3d") for N in (6, 12)]
    for c in cells:
        rate, at = c["success_within_iterations"], c["success_at_goal_within_iterations"]
        assert len(rate) == 3 and all(0.0 <= r <= 1.0 for r in rate)
        assert all(b >= a for a, b in zip(rate, rate[1:]))
        assert all(g <= r for g, r in zip(at, rate))
        assert all(np.isfinite(c["mean_reward_after_iteration"]))
    # runs of one cell use different instance ids, so their plans differ
    p, x0, goal = W.holo2d_circle(n=4, horizon=16, n_samples=128, n_steps=6)
    bc = L.BatchContext([p.replace(instance_id=j) for j in range(2)], [x0] * 2, [goal] * 2)
    bc.iterate(0)
    a, b = bc.plan_of(0).cpu().numpy(), bc.plan_of(1).cpu().numpy()
    bc.close()
    assert not np.array_equal(a, b)


def test_first_success_experiment_runs(L):
    """Time to the first conflict-free plan (the paper's headline measure):
    tiny teams are solved at once on both scenarios, within the deadline."""
    from paper_2503_12204_amd import experiments as E
    for sc in ("circle", "random"):
        print("first success", sc, "n=3 M=128 T=20 N=8, 2 runs", flush=True)
        r = E.first_success(L, scenario=sc, n=3, runs=2, n_samples=128, horizon=20, n_steps=8, radius=4.0,
                            deadline_s=5.0, max_iterations=20, log=lambda m: print(m, flush=True))
        assert r["runs"] == 2 and 0.0 <= r["solved_fraction"] <= 1.0
        assert len(r["iterations_of_solved_runs"]) == round(2 * r["solved_fraction"])
        assert all(1 <= k <= 20 for k in r["iterations_of_solved_runs"])


def test_batch_nonfinite_instance_is_flagged_alone(L):
    """An instance with a NaN goal gets status D4_ENONFINITE; its neighbours in
    the same launches keep status 0 and their single-problem results."""
    inst = _mix(3, 128, 6, seed=5, t_range=(10, 30))
    p, x0, g = inst[1]
    g = g.copy()
    g[0, 0] = np.nan
    inst[1] = (p, x0, g)
    probs = [q for q, _, _ in inst]
    print("case batch with one NaN goal", [(q.dyn, q.n_robots, q.horizon) for q in probs], flush=True)
    bc = L.BatchContext(probs, [x for _, x, _ in inst], [gg for _, _, gg in inst])
    stats = bc.iterate(0)
    got = [bc.plan_of(j).cpu().numpy() for j in range(len(probs))]
    bc.close()
    assert stats[1]["status"] == L.D4_ENONFINITE
    from paper_2503_12204_amd import autotune as AT
    for j in (0, 2):
        q, x0, g = inst[j]
        assert stats[j]["status"] == 0
        S, Tb, R = AT.get_tile(q, batched=True)
        AT.set_tile(q.dyn, q.n_robots, q.horizon, S, Tb, R)
        try:
            u, hist = L.plan(q, x0, g, iterations=1)
        finally:
            AT.clear_tile(q.dyn, q.n_robots, q.horizon)
        assert np.array_equal(u.cpu().numpy(), got[j]) and hist[0] == stats[j]


@pytest.mark.parametrize("dyn", [W.HOLO2D, W.HOLO3D, W.UNICYCLE])
def test_batch_largest_instance_against_oracle(L, dyn):
    """The largest instance shape of the 512-instance workload (32 robots, 160
    steps, 1024 samples): the fused step of the single-problem path matches
    the oracle on sampled samples (draws bit-exact, rewards and counts within
    their bars), and the same instance inside a batch reproduces that path's
    iteration bit for bit."""
    from paper_2503_12204_amd import autotune as AT
    rng = np.random.default_rng(32 + dyn)
    p, x0, g = W.random_instance(rng, dyn, 32, 160, 1024, box=10.0, min_sep=1.0)
    p = p.replace(n_steps=3, instance_id=11)
    print(f"case largest batch instance dyn={dyn} n=32 T=160 M=1024", flush=True)
    u_base = rng.uniform(-0.3, 0.3, size=p.D).astype(np.float32)
    du = (rng.normal(size=p.D) * 0.2).astype(np.float32)
    cu = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    eps, r, hits = L.sample_rollout_fitness(p, cu(x0), cu(g), cu(u_base), cu(du), 2, 3)
    torch.cuda.synchronize()
    idx = np.sort(rng.choice(p.n_samples, size=24, replace=False))
    idx[0], idx[-1] = 0, p.n_samples - 1
    ora = ombd.sample_rewards(p, x0, g, u_base, du, 2, 3, samples=idx)
    assert np.array_equal(eps.cpu().numpy()[:, idx], ora["eps"])
    from helpers import REWARD_ATOL, ambiguous_band_pairs, ambiguous_samples
    amb = ambiguous_samples(p, ora["x"])
    rg, hg = r.cpu().numpy()[idx], hits.cpu().numpy()[idx]
    ok = ~amb
    assert ok.sum() >= 6
    assert np.all(np.abs(rg[ok] - ora["r"][ok]) <= REWARD_ATOL)
    assert np.array_equal(hg[ok], ora["hits"][ok])
    assert np.all(np.abs(hg[amb] - ora["hits"][amb]) <= ambiguous_band_pairs(p, ora["x"])[amb])
    # inside a batch with a small neighbour
    q, xq, gq = _mix(1, 1024, 3, seed=9)[0]
    probs = [p, q.replace(instance_id=12)]
    bc = L.BatchContext(probs, [x0, xq], [g, gq])
    plans = [u_base.reshape(p.n_robots, p.horizon, p.du), np.zeros((q.n_robots, q.horizon, q.du), np.float32)]
    bc.set_plans(plans)
    stats = bc.iterate(0)
    got = bc.plan_of(0).cpu().numpy()
    bc.close()
    S, Tb, R = AT.get_tile(p, batched=True)
    AT.set_tile(p.dyn, p.n_robots, p.horizon, S, Tb, R)
    try:
        u, hist = L.plan(p, x0, g, iterations=1, u_init=plans[0])
    finally:
        AT.clear_tile(p.dyn, p.n_robots, p.horizon)
    assert np.array_equal(u.cpu().numpy(), got) and hist[0] == stats[0]


@pytest.mark.skip(reason="the persistent batched step did not finish on the GPU (twice, in the first batch "
                         "test, 10 instances, M = 160); the cause is not found and the form is switched off "
                         "(d4_set_option refuses it)")
def test_persistent_step_equals_two_launch_form(L):
    """The persistent step (one launch per denoising step over the work list)
    and the two-launch form (reward launch, update launch) run the same
    arithmetic on the same tiles: identical plans and statistics, graph or
    no graph, and no wait timed out (status 0)."""
    inst = _mix(20, 256, 8, seed=11, t_range=(9, 70))
    q, x0q, gq = W.diffdrive_circle(n=7, horizon=31, n_samples=256)
    inst.append((q.replace(n_steps=8, instance_id=30), x0q, gq))
    probs = [p for p, _, _ in inst]
    print("case persistent vs two-launch", len(probs), "instances", flush=True)
    res = {}
    for persistent in (1, 0):
        for graphs in (1, 0):
            with L.option("batch_persistent", persistent), L.option("graphs", graphs):
                bc = L.BatchContext(probs, [x for _, x, _ in inst], [g for _, _, g in inst])
                for it in range(2):
                    stats = bc.iterate(it)
                res[(persistent, graphs)] = (bc.u.cpu().numpy(), stats)
                bc.close()
    ref_u, ref_st = res[(0, 1)]
    assert all(s["status"] == 0 for s in ref_st)
    for key, (u, st) in res.items():
        assert np.array_equal(u, ref_u), key
        assert st == ref_st, key


def test_bucket_tiles_change_speed_only(L):
    """Tiles installed per (dynamics, team size, horizon) bucket for the
    batched form (what autotune.tune_batch installs) give the same plans and
    statistics as the rule's tiles; the tuner itself runs on a small batch,
    leaves every bucket it chose installed and the others on the rule, and a
    second call with the same batch installs the cached choice."""
    from paper_2503_12204_amd import autotune as AT
    inst = _mix(12, 128, 6, seed=13, t_range=(9, 50))
    probs = [p for p, _, _ in inst]
    print("case bucket tiles", [(p.dyn, p.n_robots, p.horizon) for p in probs], flush=True)

    def run():
        bc = L.BatchContext(probs, [x for _, x, _ in inst], [g for _, _, g in inst])
        for it in range(2):
            st = bc.iterate(it)
        u = bc.u.cpu().numpy()
        bc.close()
        return u, st

    ref_u, ref_st = run()
    buckets = sorted({AT.batch_bucket(p) for p in probs})
    try:
        for b in buckets:
            cs = 4 if b[0] == W.HOLO3D else 2
            AT.set_batch_tile(b, max(1, min(64, 256 // b[2]) // 2), 2 * cs)
        u, st = run()
        assert np.array_equal(u, ref_u) and st == ref_st
        for b in buckets:
            AT.clear_batch_tile(b)
        import tempfile
        rule = {id(p): AT.get_tile(p, batched=True) for p in probs}
        with tempfile.TemporaryDirectory() as td:
            x0s, goals = [x for _, x, _ in inst], [g for _, _, g in inst]
            chosen = AT.tune_batch(probs, x0s, goals, path=f"{td}/t.json", steps=3, min_share=0.0)
            assert set(chosen) <= set(buckets)

            def check():
                for p in probs:
                    e = chosen.get(AT.batch_bucket(p))
                    want = rule[id(p)] if e is None else (e["S"], e["Tb"], 1)
                    assert AT.get_tile(p, batched=True) == want
            check()
            u, st = run()
            assert np.array_equal(u, ref_u) and st == ref_st
            for b in buckets:
                AT.clear_batch_tile(b)
            again = AT.tune_batch(probs, x0s, goals, path=f"{td}/t.json", steps=3, min_share=0.0)
            assert {b: (e["S"], e["Tb"]) for b, e in again.items()} == {b: (e["S"], e["Tb"]) for b, e in chosen.items()}
            check()
    finally:
        for b in buckets:
            AT.clear_batch_tile(b)
