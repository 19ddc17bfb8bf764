"""Pins of the proposal network reference: finite differences, equivariance, Adam."""
import numpy as np

from oracle import proposal as P


def _small(rng):
    shapes = P.param_shapes(d_in=6, width=8, hidden=12, layers=2, d_out=5)
    params = P.init_params(rng, 6, 8, 12, 2, 5)
    for k in params:                      # non-zero biases exercise their gradients
        if params[k].ndim == 1:
            params[k] = rng.normal(size=params[k].shape) * 0.3
    seg = np.array([0, 3, 4, 9])
    x = rng.normal(size=(9, 6))
    t = rng.normal(size=(9, 5))
    mask = np.array([1, 1, 0, 1, 1, 1, 0, 1, 1], dtype=float)
    return shapes, params, seg, x, t, mask


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    shapes, params, seg, x, t, mask = _small(rng)
    y, cache = P.forward(params, x, seg, layers=2)
    L0, dy = P.loss(y, t, mask)
    grads = P.backward(params, cache, dy, layers=2)
    h = 1e-6
    for name in P.order(2):
        w = params[name]
        num = np.zeros_like(w)
        it = np.nditer(w, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            old = w[idx]
            w[idx] = old + h
            lp, _ = P.loss(P.forward(params, x, seg, 2)[0], t, mask)
            w[idx] = old - h
            lm, _ = P.loss(P.forward(params, x, seg, 2)[0], t, mask)
            w[idx] = old
            num[idx] = (lp - lm) / (2 * h)
        err = np.abs(num - grads[name]).max() / max(np.abs(num).max(), 1e-12)
        assert err < 1e-6, (name, err)


def test_permutation_equivariance():
    rng = np.random.default_rng(1)
    shapes, params, seg, x, t, mask = _small(rng)
    y, _ = P.forward(params, x, seg, 2)
    perm = np.concatenate([rng.permutation(3), 3 + rng.permutation(1), 4 + rng.permutation(5)])
    yp, _ = P.forward(params, x[perm], seg, 2)
    assert np.allclose(yp, y[perm], atol=1e-12)
    # instances do not see each other: changing one leaves the others unchanged
    x2 = x.copy()
    x2[4:9] += 1.0
    y2, _ = P.forward(params, x2, seg, 2)
    assert np.allclose(y2[:4], y[:4], atol=1e-12) and not np.allclose(y2[4:], y[4:])


def test_loss_value_and_mask():
    y = np.array([[1.0, 2.0], [0.0, 0.0], [3.0, -1.0]])
    t = np.zeros((3, 2))
    L, dy = P.loss(y, t, np.array([1.0, 1.0, 0.0]))
    assert abs(L - 5.0 / 8.0) < 1e-15      # (1 + 4) / (2 * 2 * 2)
    assert np.allclose(dy[2], 0) and np.allclose(dy[0], [0.25, 0.5])


def test_adam_first_step_closed_form():
    # after one step from zero moments, the bias-corrected step is lr * g / (|g| + eps)
    params = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -4.0, 1e-3])}
    P.adam(params, g, {}, lr=0.01)
    expect = np.array([1.0, -2.0, 0.5]) - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(params["w"], expect, rtol=0, atol=1e-15)


def test_parameter_count():
    shapes = P.param_shapes()
    n = sum(int(np.prod(s)) for s in shapes.values())
    assert n == 6 * 256 + 256 + 4 * (256 * 512 + 512 + 512 * 256 + 256 + 256 * 256) + 256 * 200 + 200
    assert 1.3e6 < n < 1.6e6


def test_bf16_rounding():
    # exactly representable values are unchanged; halfway cases go to the even neighbour
    exact = np.array([0.0, 1.0, -2.5, 1.0 + 2.0 ** -7, 2.0 ** 100, -3.0 * 2.0 ** -40])
    assert np.array_equal(P.bf16_round(exact), exact)
    assert P.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0                 # tie -> even (1.0)
    assert P.bf16_round(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6  # tie -> even (odd below)
    assert P.bf16_round(np.array([1.0 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1.0 + 2.0 ** -7
    assert P.bf16_round(np.array([-1.0 - 2.0 ** -9]))[0] == -1.0
    x = np.random.default_rng(0).normal(size=1000)
    r = P.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 + 1e-45)
    assert np.array_equal(P.bf16_round(r), r)


def test_quantised_path_is_close_and_exact_on_representable_inputs():
    rng = np.random.default_rng(4)
    shapes, params, seg, x, t, mask = _small(rng)
    y, _ = P.forward(params, x, seg, 2)
    yq, _ = P.forward(params, x, seg, 2, quant=P.bf16_round)
    assert np.abs(yq - y).max() <= 3e-2 * np.abs(y).max()
    # with identity quantisation the two paths coincide
    yi, _ = P.forward(params, x, seg, 2, quant=lambda a: a)
    assert np.array_equal(yi, y)


def test_forward_hand_computed_value():
    """One layer of width 2 (hidden 2) on two instances, worked out by hand:
    instance 0 holds robots x = (1, 0) and (0, 2), instance 1 the robot (1, 1).
    The pool averages the layer's input h_0 over the robot's own instance
    (mean over instance 0: (1.0, 0.5)); pooling the layer's output instead, or
    over all robots, changes every value below.

    h_0 = x We + be: (1.5, -0.5), (0.5, 1.5), (1.5, 0.5)
    relu(h_0 W1 + b1): (0.5, 0), (3.5, 0), (2.5, 0)
    relu(.) W2 + b2: (0.75, 1.0), (3.75, 7.0), (2.75, 5.0)
    mean(h_0) Wp: (0.5, 1.0), (0.5, 1.0), (0.5, 1.5)
    h_1: (2.75, 1.5), (4.75, 9.5), (4.75, 7.0)
    y = h_1 Wh + bh: 1.75, -4.25, -1.75
    """
    params = {
        "We": np.eye(2), "be": np.array([0.5, -0.5]),
        "W1_0": np.array([[1.0, -1.0], [2.0, 0.0]]), "b1_0": np.array([0.0, -1.0]),
        "W2_0": np.array([[1.0, 2.0], [3.0, 4.0]]), "b2_0": np.array([0.25, 0.0]),
        "Wp_0": np.array([[0.0, 1.0], [1.0, 0.0]]),
        "Wh": np.array([[1.0], [-1.0]]), "bh": np.array([0.5]),
    }
    x = np.array([[1.0, 0.0], [0.0, 2.0], [1.0, 1.0]])
    seg = np.array([0, 2, 3])
    y, cache = P.forward(params, x, seg, layers=1)
    assert np.array_equal(y[:, 0], [1.75, -4.25, -1.75])
    assert np.array_equal(cache["h"][1], [[2.75, 1.5], [4.75, 9.5], [4.75, 7.0]])
