"""What the learned proposal gains: a network trained on plans the planner
solved, judged by the planner and refined by it, against the plain planner
from zero controls on held-out teams (small scale, seconds)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_trained_proposal_beats_zero_start():
    from paper_2503_12204_amd import _lib as L
    from paper_2503_12204_amd import proposal as PR
    rng = np.random.default_rng(123)
    mk = dict(n_range=(4, 8), horizon=40, n_samples=256, n_steps=30, box=6.0)
    train = [PR.random_team(rng, instance_id=j, **mk) for j in range(160)]
    plans, hist, _ = PR.run_planner(L, train, iterations=3)
    ok = np.array([s["reward"] > 0.3 for s in hist[-1]])
    assert ok.mean() > 0.5
    prop = PR.Proposal(L, horizon=40, width=128, hidden=256, layers=2, max_rows=2048, max_batch=512, seed=3,
                       box=6.0)
    losses = prop.fit(train, plans, ok, epochs=12, batch=64, lr=2e-3)
    assert losses[-1] < losses[0]   # the plans carry sampling noise no network can predict
    test = [PR.random_team(rng, instance_id=1000 + j, **mk) for j in range(48)]
    init, used = prop.judged_initial_plans(test)
    r_net = np.array([PR.plan_reward(L, t, u) for t, u in zip(test, init)])
    assert np.mean(used) > 0.5 and r_net.mean() > 0.1      # zero controls score exactly 0 here
    _, h_plain, _ = PR.run_planner(L, test, iterations=2)
    _, h_net, _ = PR.run_planner(L, test, iterations=2, init_plans=init)
    first_plain = np.mean([s["reward"] for s in h_plain[0]])
    first_net = np.mean([s["reward"] for s in h_net[0]])
    print(f"after one iteration: plain {first_plain:.4f} proposal {first_net:.4f}", flush=True)
    assert first_net > first_plain
    prop.close()
