"""GPU parity of every C-ABI entry point against the CPU oracle.

Bars: normal draws and pair counts bit-exact; single RK4 steps within
1e-5 relative; per-sample rewards within REWARD_ATOL except samples whose
pairs sit inside the guard band of the threshold; the update within the FP32
error of the softmax and reduction; final rewards within 1e-3 relative.
"""
import numpy as np
import pytest
import torch

from helpers import (FINAL_RTOL, REWARD_ATOL, STEP_ATOL, STEP_RTOL, ambiguous_band_pairs,
                     ambiguous_obstacle_samples, ambiguous_samples, problems_small)
from oracle import dynamics as odyn
from oracle import fitness as ofit
from oracle import mbd as ombd
from oracle import noise as onoise
from oracle import schedule as osched
from paper_2503_12204_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = problems_small()
IDS = [c[0] for c in CASES]


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "the GPU tests need a HIP device"
    from paper_2503_12204_amd import _lib
    return _lib


def _cu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rand_controls(rng, p, M, spread=1.6):
    lo = np.array(p.u_lo[:p.du])
    hi = np.array(p.u_hi[:p.du])
    mid, half = (lo + hi) / 2, (hi - lo) / 2
    return (mid + half * rng.uniform(-spread, spread, size=(M, p.n_robots, p.horizon, p.du))).astype(np.float32)


@pytest.mark.parametrize("name,p,x0,g", CASES, ids=IDS)
def test_noise_bitexact(L, name, p, x0, g):
    print(f"case {name}", flush=True)
    for kappa, step in ((0, 1), (3, 100), (65535, 65535)):
        q = p.replace(seed=0xDEADBEEF12345678, instance_id=7)
        eps = _np(L.noise(q, kappa, step))
        ref = onoise.draw(q.seed, q.instance_id, kappa, step, q.n_samples, q.D)
        assert eps.dtype == np.float32
        assert np.array_equal(eps.view(np.uint32), ref.view(np.uint32)), \
            f"{int((eps != ref).sum())} of {eps.size} draws differ"


def test_box_muller_exhaustive(L):
    """Every radius word and every angle word the recipe distinguishes
    (word >> 9 takes 2^23 values each) gives the oracle's bits.  Radius words
    pair with the smallest angle (cos = 1 exactly, so z_even is rho itself);
    angle words pair with two radius words through a permutation, so sine and
    cosine show through non-trivial products."""
    print("case box-muller exhaustive", flush=True)
    j = np.arange(1 << 23, dtype=np.uint64)
    words = (j << np.uint64(9)).astype(np.uint32)
    perm = ((j * np.uint64(2654435761)) & np.uint64((1 << 23) - 1)).astype(np.uint64)
    pw = (perm << np.uint64(9)).astype(np.uint32)
    zero = np.zeros_like(words)
    for wa, wb in ((words, zero), (pw, words), (words, pw)):
        inter = np.empty(2 * wa.size, dtype=np.uint32)
        inter[0::2], inter[1::2] = wa, wb
        z = L.box_muller(torch.from_numpy(inter.view(np.int32)).cuda()).cpu().numpy()
        ze, zo = onoise.box_muller(wa.astype(np.uint64), wb.astype(np.uint64))
        assert np.array_equal(z[0::2].view(np.uint32), ze.view(np.uint32)), \
            f"{int((z[0::2] != ze).sum())} cos outputs differ"
        assert np.array_equal(z[1::2].view(np.uint32), zo.view(np.uint32)), \
            f"{int((z[1::2] != zo).sum())} sin outputs differ"


@pytest.mark.parametrize("name,p,x0,g", CASES, ids=IDS)
def test_rollout_single_step_and_trajectory(L, name, p, x0, g):
    print(f"case {name}", flush=True)
    rng = np.random.default_rng(5)
    M = min(p.n_samples, 64)
    u = _rand_controls(rng, p, M)
    x = _np(L.rollout(p, _cu(x0), _cu(u))).astype(np.float64)
    assert np.array_equal(x[:, :, 0], np.broadcast_to(x0, x[:, :, 0].shape))
    uc = odyn.clip_controls(p, u.astype(np.float64))
    for t in range(p.horizon):
        ref = odyn.step(p, x[:, :, t], uc[:, :, t])
        err = np.abs(x[:, :, t + 1] - ref)
        assert np.all(err <= STEP_RTOL * np.abs(ref) + STEP_ATOL), f"t={t} max err {err.max()}"
    # free-running trajectories: FP32 rounding accumulates over the horizon
    ref = odyn.rollout(p, x0, u)
    tol = 2e-6 * p.horizon * (1.0 + np.abs(ref).max())
    assert np.abs(x - ref).max() <= tol


@pytest.mark.parametrize("name,p,x0,g", CASES, ids=IDS)
def test_fitness_pair_counts_bitexact(L, name, p, x0, g):
    print(f"case {name}", flush=True)
    rng = np.random.default_rng(6)
    for flags in (W.FLAG_NORMALIZE, W.FLAG_SAFE_PAIRS):
        q = p.replace(flags=flags, w_safe=0.8)
        M = min(q.n_samples, 96)
        u = _rand_controls(rng, q, M)
        xg = L.rollout(q, _cu(x0), _cu(u))
        r, hits, rh = L.fitness(q, xg, _cu(g))
        x = _np(xg)
        ro, ho, rho = ofit.reward(q, x, g, pred_dtype=np.float32)
        assert np.array_equal(_np(hits), ho)
        assert np.array_equal(_np(rh), rho)
        assert np.allclose(_np(r), ro, rtol=0, atol=1e-5)


def test_fitness_sees_collisions(L):
    """A packed team guarantees hits, so the bit-exact count is exercised."""
    rng = np.random.default_rng(8)
    p, x0, g = W.random_instance(rng, W.HOLO2D, 12, 30, 128, box=3.0, min_sep=0.5)
    u = _rand_controls(rng, p, 128)
    xg = L.rollout(p, _cu(x0), _cu(u))
    r, hits, rh = L.fitness(p, xg, _cu(g))
    ro, ho, rho = ofit.reward(p, _np(xg), g, pred_dtype=np.float32)
    assert ho.sum() > 100
    assert np.array_equal(_np(hits), ho) and np.array_equal(_np(rh), rho)


@pytest.mark.parametrize("name,p,x0,g", CASES, ids=IDS)
def test_fused_step_parity(L, name, p, x0, g):
    print(f"case {name}", flush=True)
    rng = np.random.default_rng(7)
    u_base = _rand_controls(rng, p, 1, spread=0.5)[0].reshape(-1)
    du = (rng.normal(size=p.D) * 0.3).astype(np.float32)
    kappa, step = 2, 57
    eps, r, hits = L.sample_rollout_fitness(p, _cu(x0), _cu(g), _cu(u_base), _cu(du), kappa, step)
    ora = ombd.sample_rewards(p, x0, g, u_base, du, kappa, step)
    assert np.array_equal(_np(eps), ora["eps"])
    _check_rewards(p, ora, _np(r), _np(hits))


def _check_rewards(p, ora, rg, hg, min_clear=0.25):
    """Hits must match exactly wherever no pair is inside the guard band; the
    rest may differ by the pairs inside the band.  Rewards follow the same split."""
    amb = ambiguous_samples(p, ora["x"]) | ambiguous_obstacle_samples(p, ora["x"])
    ok = ~amb
    assert ok.mean() >= min_clear, f"only {ok.sum()} of {ok.size} samples clear of the guard band"
    assert np.all(np.abs(rg[ok] - ora["r"][ok]) <= REWARD_ATOL), np.abs(rg[ok] - ora["r"][ok]).max()
    assert np.array_equal(hg[ok], ora["hits"][ok])
    near = ambiguous_band_pairs(p, ora["x"])
    assert np.all(np.abs(hg[amb] - ora["hits"][amb]) <= near[amb])


def _update_tol(du_in, ms, sg, os_):
    # softmax weights carry a relative FP32 error ~ |z| 2^-24 with |z| <= ~60,
    # the weighted sum adds M roundings of a convex combination
    return 1e-4 * os_ * (sg * 4.0 + np.abs(du_in) * ms) + 1e-6


@pytest.mark.parametrize("normalize", [True, False])
@pytest.mark.parametrize("name,p,x0,g", CASES[:4], ids=IDS[:4])
def test_score_update_parity(L, name, p, x0, g, normalize):
    print(f"case {name} normalize={normalize}", flush=True)
    rng = np.random.default_rng(9)
    q = p.replace(flags=W.FLAG_NORMALIZE if normalize else 0, temperature=0.1 if normalize else 0.02)
    step = 40
    eps = L.noise(q, 1, step)
    r = (rng.normal(size=q.n_samples) * 0.05 + 0.4).astype(np.float32)
    du_in = (rng.normal(size=q.D) * 0.4).astype(np.float32)
    du_out, w = L.score_update(q, _cu(r), eps, _cu(du_in), step)
    ms, sg, os_ = osched.step_scalars(q.n_steps, q.beta_min, q.beta_max)
    ref, wref = ombd.mc_update(du_in, _np(eps), r, ms[step], sg[step], os_[step], q.temperature, normalize)
    wg = _np(w)
    assert abs(wg.astype(np.float64).sum() - 1) < 1e-5
    assert np.all(np.abs(wg - wref) <= 2e-5 * wref.max() + 1e-4 * wref)
    assert np.all(np.abs(_np(du_out) - ref) <= _update_tol(du_in, ms[step], sg[step], os_[step]))


@pytest.mark.parametrize("M", [4, 128, 256, 260, 1024, 1028, 16384])
def test_score_update_forms_at_their_boundaries(L, M):
    """The update kernel's forms around their boundaries: the one-wave form
    (M <= 256, a multiple of 4), the four-wave register form (J = 1 and 2)
    and, at 1028, two float4 columns for some lanes and one for others;
    each against the oracle's weighted update (Eqs. mc, mbd-denoising), with
    every row of a range that is not a multiple of the rows per pass; 16384,
    the largest sample count one workgroup's weights cover, takes sixteen
    columns per lane."""
    print(f"case update forms M={M}", flush=True)
    q, _, _ = W.holo2d_circle(n=3, horizon=9, n_samples=M)
    rng = np.random.default_rng(M)
    step = 7
    eps = L.noise(q, 2, step)
    r = (rng.normal(size=M) * 0.05 + 0.4).astype(np.float32)
    du_in = (rng.normal(size=q.D) * 0.4).astype(np.float32)
    du_out, w = L.score_update(q, _cu(r), eps, _cu(du_in), step)
    ms, sg, os_ = osched.step_scalars(q.n_steps, q.beta_min, q.beta_max)
    ref, wref = ombd.mc_update(du_in, _np(eps), r, ms[step], sg[step], os_[step], q.temperature, True)
    wg = _np(w)
    assert abs(wg.astype(np.float64).sum() - 1) < 1e-5
    assert np.all(np.abs(wg - wref) <= 2e-5 * wref.max() + 1e-4 * wref)
    assert np.all(np.abs(_np(du_out) - ref) <= _update_tol(du_in, ms[step], sg[step], os_[step]))


def test_score_update_refuses_more_samples_than_a_workgroup_weights(L):
    """Above 16384 samples the update is refused (D4_EUNSUPPORTED) before any launch."""
    q, _, _ = W.holo2d_circle(n=2, horizon=3, n_samples=16388)
    eps = torch.zeros((q.D, q.n_samples), device="cuda")
    with pytest.raises(L.D4Error) as e:
        L.score_update(q, torch.zeros(q.n_samples, device="cuda"), eps, torch.zeros(q.D, device="cuda"), 1)
    assert e.value.code == L.D4_EUNSUPPORTED


def test_score_update_degenerate_rewards(L):
    p, x0, g = W.holo2d_circle(n=4, horizon=10, n_samples=200)
    eps = L.noise(p, 0, 5)
    du_in = np.linspace(-1, 1, p.D).astype(np.float32)
    du_out, w = L.score_update(p, _cu(np.full(200, 0.25, np.float32)), eps, _cu(du_in), 5)
    assert np.allclose(_np(w), 1 / 200, rtol=1e-6)
    ms, sg, os_ = osched.step_scalars(p.n_steps, p.beta_min, p.beta_max)
    ref, _ = ombd.mc_update(du_in, _np(eps), np.full(200, 0.25), ms[5], sg[5], os_[5], p.temperature)
    assert np.all(np.abs(_np(du_out) - ref) <= _update_tol(du_in, ms[5], sg[5], os_[5]))


def _gpu_iteration_stepwise(L, p, x0, g, u_base, kappa, check_steps, ora_checks):
    """Run one iteration through the split entry points, checking chosen steps
    against the oracle fed the GPU's own Delta U_i and rewards."""
    ms, sg, os_ = osched.step_scalars(p.n_steps, p.beta_min, p.beta_max)
    du = torch.zeros(p.D, dtype=torch.float32, device="cuda")
    x0c, gc, ubc = _cu(x0), _cu(g), _cu(u_base.reshape(-1))
    for i in range(p.n_steps, 0, -1):
        eps, r, hits = L.sample_rollout_fitness(p, x0c, gc, ubc, du, kappa, i)
        du_next, w = L.score_update(p, r, eps, du, i)
        if i in check_steps:
            dui = _np(du)
            ora = ombd.sample_rewards(p, x0, g, u_base.reshape(-1), dui, kappa, i)
            assert np.array_equal(_np(eps), ora["eps"]), f"step {i}"
            rg = _np(r)
            _check_rewards(p, ora, rg, _np(hits))
            ref, _ = ombd.mc_update(dui, ora["eps"], rg, ms[i], sg[i], os_[i], p.temperature,
                                    bool(p.flags & W.FLAG_NORMALIZE))
            assert np.all(np.abs(_np(du_next) - ref) <= _update_tol(dui, ms[i], sg[i], os_[i])), f"step {i}"
            ora_checks.append(i)
        du = du_next
    return du


def test_denoise_iteration_chain_and_graph(L):
    """Config 0 in full: teacher-forced chain through the split calls, then the
    graph-replayed d4_denoise_iter must reproduce the split calls bit for bit,
    and its final reward must match the oracle's for the same plan."""
    p, x0, g = W.holo2d_circle()
    rng = np.random.default_rng(4)
    u_base = _rand_controls(rng, p, 1, spread=0.3)[0]
    kappa = 1
    checks = []
    du0 = _gpu_iteration_stepwise(L, p, x0, g, u_base, kappa,
                                  {100, 99, 90, 75, 50, 25, 10, 2, 1}, checks)
    assert len(checks) == 9
    lo, hi = np.array(p.u_lo[:2], np.float32), np.array(p.u_hi[:2], np.float32)
    u_expect = np.minimum(np.maximum(u_base + _np(du0).reshape(u_base.shape), lo), hi)
    for graphs in (0, 1):
        with L.option("graphs", graphs):
            ctx = L.Context(p)
            u = _cu(u_base)
            traj = torch.empty((p.n_robots, p.horizon + 1, p.dx), dtype=torch.float32, device="cuda")
            st = ctx.denoise_iter(_cu(x0), _cu(g), u, kappa, traj=traj)
            ctx.close()
        assert st["status"] == 0
        assert np.array_equal(_np(u), u_expect), f"graphs={graphs}"
        fin = ombd.apply_deformation(p, x0, g, u_base, _np(du0))
        assert abs(st["reward"] - fin["r"]) <= FINAL_RTOL * abs(fin["r"])
        assert st["hits"] == fin["hits"] and st["success"] == fin["success"]
        assert st["at_goal"] == fin["at_goal"]
        assert abs(st["objective"] - fin["objective"]) < 1e-6  # FP32 ratio of counts
        assert np.allclose(_np(traj), fin["x"], rtol=0, atol=2e-6 * p.horizon * 5)


def test_graph_recaptures_on_changed_scalars(L):
    p, x0, g = W.holo2d_circle(n=4, horizon=20, n_samples=128)
    p = p.replace(n_steps=10)
    ctx = L.Context(p)
    res = {}
    for seed in (0, 1, 0):
        q = p.replace(seed=seed)
        u = torch.zeros((4, 20, 2), dtype=torch.float32, device="cuda")
        ctx.denoise_iter(_cu(x0), _cu(g), u, 0, p=q)
        res.setdefault(seed, []).append(_np(u))
    ctx.close()
    assert np.array_equal(res[0][0], res[0][1])
    assert not np.array_equal(res[0][0], res[1][0])


def test_free_running_iteration_matches_oracle(L):
    """One full iteration on the 4-robot circle swap, GPU and oracle each running
    on its own.  The two chains see the same draws but FP32 and FP64 rewards;
    with a near-argmax softmax (lambda = 0.1 on z-scores) a tie broken
    differently sends the chains down different, equally valid paths, so only a
    distribution-level agreement is asserted here; step-level parity is the
    teacher-forced chain above."""
    p, x0, g = W.holo2d_circle()
    u = torch.zeros((p.n_robots, p.horizon, p.du), dtype=torch.float32, device="cuda")
    ctx = L.Context(p)
    st = ctx.denoise_iter(_cu(x0), _cu(g), u, 0)
    ctx.close()
    ora = ombd.denoise_iteration(p, x0, g, np.zeros((p.n_robots, p.horizon, p.du)), 0)
    print(f"gpu reward {st['reward']:.6f} oracle {ora['r']:.6f}", flush=True)
    assert abs(st["reward"] - ora["r"]) <= 0.05 * abs(ora["r"])
    assert st["reward"] > 0.4 and ora["r"] > 0.4   # zero controls score 0


@pytest.mark.parametrize("which", ["holo3d_sphere_16x100x8192", "unicycle_8x100x2048"])
def test_full_size_sampled(L, which):
    """Full configuration sizes in the launch shape the bench times: sampled
    samples against the oracle, and sampled rows of the update."""
    if which.startswith("holo3d"):
        p, x0, g = W.holo3d_sphere()
    else:
        p, x0, g = W.unicycle_random()
    print(f"case {which}", flush=True)
    rng = np.random.default_rng(12)
    u_base = _rand_controls(rng, p, 1, spread=0.3)[0].reshape(-1)
    du = (rng.normal(size=p.D) * 0.2).astype(np.float32)
    kappa, step = 4, 100
    eps, r, hits = L.sample_rollout_fitness(p, _cu(x0), _cu(g), _cu(u_base), _cu(du), kappa, step)
    idx = np.sort(rng.choice(p.n_samples, size=48, replace=False))
    idx[0], idx[-1] = 0, p.n_samples - 1
    ora = ombd.sample_rewards(p, x0, g, u_base, du, kappa, step, samples=idx)
    eg = _np(eps)
    assert np.array_equal(eg[:, idx], ora["eps"])
    _check_rewards(p, ora, _np(r)[idx], _np(hits)[idx])
    du_out, w = L.score_update(p, r, eps, _cu(du), step)
    ms, sg, os_ = osched.step_scalars(p.n_steps, p.beta_min, p.beta_max)
    wref = ombd.weights(_np(r), p.temperature, True)
    rows = np.sort(rng.choice(p.D, size=64, replace=False))
    samples_rows = du[rows, None] * ms[step] + sg[step] * eg[rows].astype(np.float64)
    ref = os_[step] * (samples_rows * wref[None, :]).sum(1)
    assert np.all(np.abs(_np(du_out)[rows] - ref) <= _update_tol(du[rows], ms[step], sg[step], os_[step]))
    assert abs(_np(w).astype(np.float64).sum() - 1) < 1e-5


def test_invalid_arguments_raise(L):
    p, x0, g = W.holo2d_circle()
    with pytest.raises(L.D4Error):
        L.noise(p.replace(n_robots=0), 0, 1)
    with pytest.raises(L.D4Error):
        L.noise(p, 0, 0)
    with pytest.raises(L.D4Error):
        L.score_update(p, torch.zeros(p.n_samples, device="cuda"), torch.zeros((p.D, p.n_samples), device="cuda"),
                       torch.zeros(p.D, device="cuda"), p.n_steps + 1)
    with pytest.raises(L.D4Error):
        L.Context(p.replace(temperature=0.0))


def test_phase_free_and_general_draw_windows_agree(L):
    """The phase-0 draw window (T d_u a multiple of 4) and the general window
    produce the same draws, rewards and counts."""
    p, x0, g = W.holo3d_sphere(n=8, horizon=40, n_samples=256)
    rng = np.random.default_rng(2)
    ub = _cu(_rand_controls(rng, p, 1, spread=0.5)[0].reshape(-1))
    du = _cu((rng.normal(size=p.D) * 0.3).astype(np.float32))
    outs = []
    for aligned in (1, 0):
        with L.option("aligned_draws", aligned):
            outs.append([_np(t) for t in L.sample_rollout_fitness(p, _cu(x0), _cu(g), ub, du, 1, 33)])
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.allclose(outs[0][1], outs[1][1], rtol=0, atol=1e-6)
    assert np.array_equal(outs[0][2], outs[1][2])


def test_autotuned_tile_keeps_parity(L, tmp_path):
    """A tuned tile changes speed, not the method: draws stay bit-exact and the
    chain still meets the bar; the cache round-trips."""
    from paper_2503_12204_amd import autotune as AT
    p, x0, g = W.unicycle_random(n=8, horizon=40, n_samples=512)
    path = str(tmp_path / "tiles.json")
    e = AT.tune(p, x0, g, path=path, reps=2)
    assert 1 <= e["S"] <= 64 and e["Tb"] % 2 == 0 and e["us"] > 0
    try:
        assert AT.tune(p, x0, g, path=path) == e   # served from the cache
        assert AT.install_cache(path) == 1
        rng = np.random.default_rng(3)
        ub = _rand_controls(rng, p, 1, spread=0.5)[0].reshape(-1)
        du = (rng.normal(size=p.D) * 0.3).astype(np.float32)
        eps, r, hits = L.sample_rollout_fitness(p, _cu(x0), _cu(g), _cu(ub), _cu(du), 0, 50)
        ora = ombd.sample_rewards(p, x0, g, ub, du, 0, 50)
        assert np.array_equal(_np(eps), ora["eps"])
        _check_rewards(p, ora, _np(r), _np(hits))
    finally:
        AT.clear_tile(p.dyn, p.n_robots, p.horizon)


@pytest.mark.parametrize("dyn,n,T,M,S,Tb", [(W.UNICYCLE, 8, 100, 2048, 8, 16), (W.HOLO3D, 5, 37, 77, 8, 8),
                                           (W.HOLO2D, 3, 41, 50, 16, 6), (W.HOLO3D, 16, 20, 40, 4, 4),
                                           (W.DIFFDRIVE, 6, 31, 90, 8, 8)])
def test_cooperative_kernel_is_bit_identical(L, dyn, n, T, M, S, Tb):
    """Replica lanes sharing the draws and pair checks reproduce the one-lane
    kernel exactly: draws, rewards, hit counts and a whole iteration."""
    from paper_2503_12204_amd import autotune as AT
    rng = np.random.default_rng(n * T)
    p, x0, g = W.random_instance(rng, dyn, n, T, M, box=max(3.0, n ** 0.5 * 1.5), min_sep=0.6)
    p = p.replace(n_steps=6)
    ub = _cu(_rand_controls(rng, p, 1, spread=0.5)[0].reshape(-1))
    du = _cu((rng.normal(size=p.D) * 0.3).astype(np.float32))
    outs, plans = [], []
    try:
        for R in (1, 2, 4, 8, 16):
            if R * S * n > 1024:
                continue
            AT.set_tile(p.dyn, n, T, S, Tb, R)
            outs.append([_np(t) for t in L.sample_rollout_fitness(p, _cu(x0), _cu(g), ub, du, 3, 5)])
            ctx = L.Context(p)
            u = torch.zeros((n, T, p.du), dtype=torch.float32, device="cuda")
            ctx.denoise_iter(_cu(x0), _cu(g), u, 0)
            ctx.close()
            plans.append(_np(u))
    finally:
        AT.clear_tile(p.dyn, n, T)
    assert len(outs) >= 2
    for o, pl in zip(outs[1:], plans[1:]):
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
        assert np.array_equal(plans[0], pl)


@pytest.mark.parametrize("dyn,n,T,S,Tb,n_obs", [
    (W.HOLO2D, 4, 45, 16, 8, 0),      # pipelined (n S = 64), ragged last block
    (W.DIFFDRIVE, 8, 100, 8, 20, 0),  # pipelined, the c2 shape with the second heading model
    (W.UNICYCLE, 8, 33, 8, 34, 0),    # pipelined with a single time block
    (W.HOLO2D, 8, 50, 8, 12, 3),      # pipelined with obstacles (goal and obstacle terms on replica 1)
    (W.HOLO3D, 8, 41, 8, 12, 2),      # pipelined 3D with obstacles, ragged
    (W.UNICYCLE, 5, 47, 8, 10, 2),    # sequential (n S = 40) with obstacles
    (W.HOLO3D, 16, 30, 8, 8, 0),      # pipelined over two waves of replica 0 (n S = 128)
])
def test_cooperative_schedules_match_one_lane_kernel(L, dyn, n, T, S, Tb, n_obs):
    """Both schedules of the cooperative kernel (pipelined when replica 0 fills
    whole waves, sequential otherwise), for R = 2 (one replica does the
    draws, pairs, goal terms and masks), R = 3 (scorer and one worker) and up
    to 16, with one or several time blocks, a ragged last block and
    obstacles: draws, rewards, hit counts and a whole iteration equal the
    one-lane kernel's bit for bit."""
    from paper_2503_12204_amd import autotune as AT
    rng = np.random.default_rng(7 * n + T + n_obs)
    obs = tuple((rng.uniform(-1.0, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(-0.5, 0.5), 0.25) for _ in range(n_obs))
    M = 96
    p, x0, g = W.random_instance(rng, dyn, n, T, M, box=max(3.0, n ** 0.5 * 1.5), min_sep=0.6, obstacles=obs)
    p = p.replace(n_steps=5)
    ub = _cu(_rand_controls(rng, p, 1, spread=0.5)[0].reshape(-1))
    du = _cu((rng.normal(size=p.D) * 0.3).astype(np.float32))
    runs = {}
    try:
        for R in (1, 2, 3, 4, 16):
            if R * S * n > 1024:
                continue
            print("cooperative schedule case", W.DYN_NAMES[dyn], n, T, S, Tb, R, n_obs, flush=True)
            AT.set_tile(p.dyn, n, T, S, Tb, R)
            step = [_np(t) for t in L.sample_rollout_fitness(p, _cu(x0), _cu(g), ub, du, 2, 4)]
            ctx = L.Context(p)
            u = torch.zeros((n, T, p.du), dtype=torch.float32, device="cuda")
            st = ctx.denoise_iter(_cu(x0), _cu(g), u, 0)
            ctx.close()
            runs[R] = (step, _np(u), st)
    finally:
        AT.clear_tile(p.dyn, n, T)
    assert 1 in runs and len(runs) >= 3
    ref_step, ref_u, ref_st = runs[1]
    for R, (step, u, st) in runs.items():
        for a, b in zip(ref_step, step):
            assert np.array_equal(a, b), f"R = {R}"
        assert np.array_equal(u, ref_u), f"R = {R}"
        assert st == ref_st, f"R = {R}"


def test_negative_rewards_in_partial_waves(L):
    """A packed 3-robot team (collision penalties make rewards negative) with
    workgroups smaller than a wave: the split calls reproduce the graph
    iteration bit for bit (the batch statistics include the maximum of
    all-negative rewards)."""
    rng = np.random.default_rng(21)
    p, x0, g = W.random_instance(rng, W.HOLO2D, 3, 30, 70, box=1.6, min_sep=0.5)
    p = p.replace(n_steps=8, w_safe=3.0)
    u_base = _rand_controls(rng, p, 1, spread=0.2)[0]
    eps, r, _ = L.sample_rollout_fitness(p, _cu(x0), _cu(g), _cu(u_base.reshape(-1)),
                                         torch.zeros(p.D, device="cuda"), 0, 8)
    assert (_np(r) < 0).all()
    du0 = _gpu_iteration_stepwise(L, p, x0, g, u_base, 0, set(), [])
    lo, hi = np.array(p.u_lo[:2], np.float32), np.array(p.u_hi[:2], np.float32)
    expect = np.minimum(np.maximum(u_base + _np(du0).reshape(u_base.shape), lo), hi)
    ctx = L.Context(p)
    u = _cu(u_base)
    ctx.denoise_iter(_cu(x0), _cu(g), u, 0)
    ctx.close()
    assert np.array_equal(_np(u), expect)


@pytest.mark.parametrize("dyn,n,T,M", [(W.HOLO3D, 7, 23, 301), (W.UNICYCLE, 12, 40, 256), (W.HOLO2D, 2, 9, 64),
                                       (W.DIFFDRIVE, 9, 28, 200)])
def test_tile_does_not_change_results(L, dyn, n, T, M):
    """Samples per workgroup, time block and replica lanes change speed only:
    a whole iteration gives the same bits for every admissible tile."""
    from paper_2503_12204_amd import autotune as AT
    rng = np.random.default_rng(n + T)
    p, x0, g = W.random_instance(rng, dyn, n, T, M, box=max(3.0, n ** 0.5 * 1.5), min_sep=0.6)
    p = p.replace(n_steps=5)
    u0 = _rand_controls(rng, p, 1, spread=0.5)[0]
    cs = 4 if p.du == 3 else 2
    tiles = [(1, cs, 1), (3, 2 * cs, 1), (min(64, 256 // n), 4 * cs, 1), (2, 4 * cs, 2), (4, cs, 4), (1, 2 * cs, 8), (1, cs, 16)]
    plans = []
    for S, Tb, R in tiles:
        if S * n > 256 or R * S * n > 1024:
            continue
        AT.set_tile(p.dyn, p.n_robots, p.horizon, S, Tb, R)
        try:
            ctx = L.Context(p)
            u = _cu(u0)
            st = ctx.denoise_iter(_cu(x0), _cu(g), u, 0)
            ctx.close()
        finally:
            AT.clear_tile(p.dyn, p.n_robots, p.horizon)
        plans.append((S, Tb, R, _np(u), st["reward"]))
    assert len(plans) >= 3
    for S, Tb, R, u, rew in plans[1:]:
        assert np.array_equal(u, plans[0][3]), f"tile {(S, Tb, R)}"
        assert rew == plans[0][4]


@pytest.mark.parametrize("n_obs", [1, 4])
def test_final_stats_with_obstacles(L, n_obs):
    """The iteration's final scoring with obstacles (appendix penalty): on the
    GPU's own FP32 trajectory the oracle's FP32 predicates give the same pair
    hits, obstacle hits and success, and the same reward within FP32 sums."""
    p, x0, g = W.holo2d_circle_obstacles(n=8, n_obs=n_obs, horizon=40, n_samples=256)
    p = p.replace(n_steps=20)
    ctx = L.Context(p)
    u = torch.zeros((p.n_robots, p.horizon, p.du), dtype=torch.float32, device="cuda")
    traj = torch.empty((p.n_robots, p.horizon + 1, p.dx), dtype=torch.float32, device="cuda")
    for it in range(2):
        st = ctx.denoise_iter(_cu(x0), _cu(g), u, it, traj=traj)
    ctx.close()
    x = _np(traj)[None]
    r, hits, _ = ofit.reward(p, x, g, pred_dtype=np.float32)
    assert st["hits"] == int(hits[0])
    assert st["obstacle_hits"] == int(ofit.obstacle_hits(p, x, pred_dtype=np.float32).sum())
    assert abs(st["reward"] - r[0]) <= 1e-5
    assert st["success"] == bool(ofit.success(p, x.astype(np.float64), g)[0])
    assert st["at_goal"] == bool(ofit.at_goal(p, x.astype(np.float64), g)[0])


def test_obstacles_are_avoided(L):
    """A robot crossing the centre plans around a large central obstacle:
    without the penalty the straight line runs through it."""
    p, x0, g = W.holo2d_circle_obstacles(n=2, n_obs=1, horizon=60, n_samples=1024)
    plain = p.replace(obstacles=())
    out = {}
    for name, q in (("with", p), ("without", plain)):
        u, hist = L.plan(q, x0, g, iterations=3)
        x = _np(L.rollout(p, _cu(x0), u[None].contiguous()))
        out[name] = int(ofit.obstacle_hits(p, x, pred_dtype=np.float32).sum())
    assert out["without"] > 0
    assert out["with"] == 0


def test_sixteen_obstacles_with_tiny_workgroups(L):
    """Obstacle staging with workgroups smaller than the obstacle count (one
    sample of two robots is two lanes): every tile sees all 16 obstacles, so
    every tile gives the same plan and reward."""
    from paper_2503_12204_amd import autotune as AT
    rng = np.random.default_rng(16)
    obs = tuple((0.4 + 0.75 * (i % 4), 0.4 + 0.75 * (i // 4), 0.0, 0.15) for i in range(16))
    p, x0, g = W.random_instance(rng, W.HOLO2D, 2, 30, 64, box=3.0, min_sep=0.8, obstacles=obs)
    p = p.replace(n_steps=5)
    assert len(p.obstacles) == 16
    plans = []
    for S, Tb, R in [(32, 8, 1), (1, 2, 1), (2, 4, 1), (1, 2, 4)]:
        AT.set_tile(p.dyn, p.n_robots, p.horizon, S, Tb, R)
        try:
            print("16 obstacles, tile", (S, Tb, R), flush=True)
            ctx = L.Context(p)
            u = torch.zeros((p.n_robots, p.horizon, p.du), dtype=torch.float32, device="cuda")
            st = ctx.denoise_iter(_cu(x0), _cu(g), u, 0)
            ctx.close()
        finally:
            AT.clear_tile(p.dyn, p.n_robots, p.horizon)
        plans.append((S, Tb, R, _np(u), st["reward"], st["obstacle_hits"]))
    for S, Tb, R, u, rew, oh in plans[1:]:
        assert np.array_equal(u, plans[0][3]), f"tile {(S, Tb, R)}"
        assert rew == plans[0][4] and oh == plans[0][5]


@pytest.mark.parametrize("dyn", [W.UNICYCLE, W.DIFFDRIVE])
def test_late_horizon_heading(L, dyn):
    """160 steps turning at the control bound: the unwrapped heading reaches
    about 16 pi.  Every single step, from the GPU's own state, stays within
    the step bar (Sec. V models), and the fused step's draws and rewards meet
    their bars at that horizon."""
    rng = np.random.default_rng(160 + dyn)
    p, x0, g = W.random_instance(rng, dyn, 6, 160, 64, box=5.0, min_sep=0.8)
    print(f"case late heading dyn={dyn} n=6 T=160 M=64", flush=True)
    om = 1 if dyn == W.UNICYCLE else 0   # index of omega in u
    u = _rand_controls(rng, p, p.n_samples, spread=0.9)
    u[..., om] = np.float32(p.u_hi[om]) * rng.uniform(0.9, 1.2, size=u.shape[:-1]).astype(np.float32)
    x = _np(L.rollout(p, _cu(x0), _cu(u))).astype(np.float64)
    assert np.abs(x[:, :, -1, 2]).max() > 14 * np.pi
    uc = odyn.clip_controls(p, u.astype(np.float64))
    for t in range(p.horizon):
        ref = odyn.step(p, x[:, :, t], uc[:, :, t])
        err = np.abs(x[:, :, t + 1] - ref)
        assert np.all(err <= STEP_RTOL * np.abs(ref) + STEP_ATOL), f"t={t} max err {err.max()}"
    ref = odyn.rollout(p, x0, u)
    assert np.abs(x - ref).max() <= 2e-6 * p.horizon * (1.0 + np.abs(ref).max())
    # fused step: the plan turns at the bound, the draws add sigma_i eps
    ub = np.zeros((p.n_robots, p.horizon, p.du), np.float32)
    ub[..., om] = np.float32(p.u_hi[om])
    ub = ub.reshape(-1)
    du = (rng.normal(size=p.D) * 0.1).astype(np.float32)
    eps, r, hits = L.sample_rollout_fitness(p, _cu(x0), _cu(g), _cu(ub), _cu(du), 1, 30)
    ora = ombd.sample_rewards(p, x0, g, ub, du, 1, 30)
    assert np.abs(ora["x"][:, :, -1, 2]).max() > 14 * np.pi
    assert np.array_equal(_np(eps), ora["eps"])
    _check_rewards(p, ora, _np(r), _np(hits))


def test_nonfinite_reward_sets_status(L):
    """A NaN goal makes every reward non-finite: the update kernels set the
    iteration's status to D4_ENONFINITE (the non-finite check of the batch
    statistics) and every kernel still runs to completion, so the same
    context then runs the finite problem with status 0 and the plan of a
    fresh context."""
    p, x0, g = W.holo2d_circle(n=4, horizon=20, n_samples=128)
    p = p.replace(n_steps=8)
    bad = g.copy()
    bad[1, 0] = np.nan
    print("case non-finite goal n=4 T=20 M=128 N=8", flush=True)
    ctx = L.Context(p)
    u = torch.zeros((p.n_robots, p.horizon, p.du), dtype=torch.float32, device="cuda")
    st = ctx.denoise_iter(_cu(x0), _cu(bad), u, 0)
    assert st["status"] == L.D4_ENONFINITE
    assert not np.isfinite(st["reward"])
    u = torch.zeros_like(u)
    st = ctx.denoise_iter(_cu(x0), _cu(g), u, 0)
    ctx.close()
    assert st["status"] == 0 and np.isfinite(st["reward"])
    ctx = L.Context(p)
    u2 = torch.zeros_like(u)
    st2 = ctx.denoise_iter(_cu(x0), _cu(g), u2, 0)
    ctx.close()
    assert np.array_equal(_np(u), _np(u2)) and st == st2
    # the split update call flags nothing but still yields finite uniform weights
    eps = L.noise(p, 0, 3)
    r = torch.full((p.n_samples,), float("nan"), device="cuda")
    du_out, w = L.score_update(p, r, eps, torch.zeros(p.D, device="cuda"), 3)
    assert np.allclose(_np(w), 1.0 / p.n_samples, rtol=1e-6)
    assert np.isfinite(_np(du_out)).all()
