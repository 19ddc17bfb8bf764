"""The persistent batched step's work list and its queue semantics, on the
CPU (the list is built by the library's host code, d4_batch_work_list).

Every reward tile of an instance comes before every update tile of it, so a
workgroup that takes an update tile waits only on reward tiles that running
workgroups already hold: a simulation of any number of workgroups taking
items in order, each update tile blocking until its instance's reward tiles
have finished, always drains the list."""
import heapq

import numpy as np
import pytest

from paper_2503_12204_amd import workloads as W


@pytest.fixture(scope="module")
def L():
    from paper_2503_12204_amd import _lib
    return _lib


def _mix(count, M, seed=0, **kw):
    return [p for p, _, _ in W.batched_mix(count=count, n_samples=M, seed=seed, **kw)]


def _check_list(L, probs, items, lag):
    from paper_2503_12204_amd import autotune as AT
    M = probs[0].n_samples
    kinds, inst, a, b = items.T
    assert set(np.unique(kinds)) <= {0, 1}
    last_reward = {}
    first_update = {}
    for pos, (k, j) in enumerate(zip(kinds, inst)):
        if k == 0:
            last_reward[j] = pos
        else:
            first_update.setdefault(j, pos)
    for j, p in enumerate(probs):
        S = AT.get_tile(p, batched=True)[0]
        m0 = np.sort(a[(kinds == 0) & (inst == j)])
        assert np.array_equal(m0, np.arange(0, M, S)), f"reward tiles of instance {j}"
        rows = sorted(zip(a[(kinds == 1) & (inst == j)], b[(kinds == 1) & (inst == j)]))
        assert rows[0][0] == 0 and rows[-1][1] == p.D and all(x[1] == y[0] for x, y in zip(rows, rows[1:]))
        assert all(0 < e1 - e0 <= 64 for e0, e1 in rows)
        assert last_reward[j] < first_update[j], f"instance {j}: an update tile precedes a reward tile"
    # the lag: an instance's update tiles wait for `lag` further reward tiles, unless the list ran out of them
    reward_pos = np.flatnonzero(kinds == 0)
    for j in range(len(probs)):
        later = np.count_nonzero((reward_pos > last_reward[j]) & (reward_pos < first_update[j]))
        remaining = np.count_nonzero(reward_pos > last_reward[j])
        assert later >= min(lag, remaining), (j, later, remaining)


@pytest.mark.parametrize("lag", [0, 7, 512])
def test_work_list_of_the_512_instance_mix(L, lag):
    probs = _mix(512, 1024)
    items = L.batch_work_list(probs, lag)
    _check_list(L, probs, items, lag)
    # instances in descending tile cost: the largest work comes first
    assert items[0][0] == 0


def test_work_list_small_and_degenerate(L):
    probs = _mix(5, 70, seed=3, n_range=(1, 6), t_range=(1, 9))
    for lag in (0, 1, 1000):
        _check_list(L, probs, L.batch_work_list(probs, lag), lag)
    one = _mix(1, 1, seed=4)
    items = L.batch_work_list(one, 3)
    assert items[0][0] == 0 and (items[1:, 0] == 1).all()


def _simulate(items, tiles_of, workers, rng):
    """Workers take items in list order; an update item blocks (polling) until
    its instance's reward tiles have finished.  Returns the finish time and the
    largest number of polls any wait took."""
    done = np.zeros(len(tiles_of), dtype=np.int64)
    t_free = [(0.0, w) for w in range(workers)]
    heapq.heapify(t_free)
    finish_events = []            # (time, instance) of reward tiles finishing
    nxt, max_polls, now = 0, 0, 0.0
    while nxt < len(items):
        now, w = heapq.heappop(t_free)
        kind, j, _, _ = items[nxt]
        nxt += 1
        while finish_events and finish_events[0][0] <= now:
            _, jj = heapq.heappop(finish_events)
            done[jj] += 1
        if kind == 0:
            end = now + rng.uniform(0.5, 3.0)
            heapq.heappush(finish_events, (end, j))
        else:
            polls = 0
            while done[j] < tiles_of[j]:
                assert finish_events, "update tile waits on a reward tile nobody holds"
                now, jj = heapq.heappop(finish_events)
                done[jj] += 1
                polls += 1
            max_polls = max(max_polls, polls)
            end = now + rng.uniform(0.2, 1.0)
        heapq.heappush(t_free, (end, w))
    return max(t for t, _ in t_free), max_polls


@pytest.mark.parametrize("workers", [1, 2, 13, 512])
def test_queue_always_drains(L, workers):
    from paper_2503_12204_amd import autotune as AT
    probs = _mix(24, 256, seed=9)
    items = L.batch_work_list(probs, workers)
    tiles_of = np.array([-(-p.n_samples // AT.get_tile(p, batched=True)[0]) for p in probs])
    assert np.array_equal(np.bincount(items[items[:, 0] == 0, 1], minlength=len(probs)), tiles_of)
    rng = np.random.default_rng(workers)
    t_end, max_polls = _simulate(items, tiles_of, workers, rng)
    assert np.isfinite(t_end)
    # a wait never outlasts the reward tiles already taken
    assert max_polls <= tiles_of.max() * len(probs)
