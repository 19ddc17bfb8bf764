"""FP64 reference of the learned proposal network (test infrastructure).

The learned proposal predicts the initial plan tau.u that Algorithm 2 starts
from (the paper initialises tau without learning; the proposal replaces that
initialisation, and the plain planner still judges and refines its output).
The network is permutation-equivariant over the robots of one instance:

  h_0 = x W_e + b_e                                    x: per-robot features
  h_{l+1} = h_l + relu(h_l W1_l + b1_l) W2_l + b2_l + mean_b(h_l) Wp_l
  y = h_L W_h + b_h                                    y: per-robot controls [T d_u]

where mean_b averages the rows of the robot's own instance.  Loss:
L = sum_r mask_r |y_r - t_r|^2 / (2 d_out sum_r mask_r).  Optimiser: Adam
(Kingma and Ba, 2015) with bias correction.

Every function is plain NumPy in FP64; the backward pass is written out by
hand.  With `quant=bf16_round` every operand of a matrix product (activations,
pooled rows, upstream gradients) is rounded to BF16 first, as a BF16 product
kernel sees it; the products themselves stay exact, so ReLU gates and losses
are decided at the kernel's operand precision.  Pinned by central finite
differences of the loss against every parameter tensor, permutation
equivariance, Adam's closed-form first step and BF16 rounding of exactly
representable and midpoint values (tests/test_oracle_proposal.py).
"""
import numpy as np


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(a):
    return a


def param_shapes(d_in=6, width=256, hidden=512, layers=4, d_out=200):
    shapes = {"We": (d_in, width), "be": (width,)}
    for l in range(layers):
        shapes[f"W1_{l}"] = (width, hidden)
        shapes[f"b1_{l}"] = (hidden,)
        shapes[f"W2_{l}"] = (hidden, width)
        shapes[f"b2_{l}"] = (width,)
        shapes[f"Wp_{l}"] = (width, width)
    shapes["Wh"] = (width, d_out)
    shapes["bh"] = (d_out,)
    return shapes


def order(layers=4):
    return ["We", "be"] + [f"{n}{l}" for l in range(layers) for n in ("W1_", "b1_", "W2_", "b2_", "Wp_")] + ["Wh", "bh"]


def init_params(rng, d_in=6, width=256, hidden=512, layers=4, d_out=200):
    """Uniform(+-1/sqrt(fan_in)) weights, zero biases."""
    out = {}
    for name, shp in param_shapes(d_in, width, hidden, layers, d_out).items():
        if len(shp) == 1:
            out[name] = np.zeros(shp)
        else:
            lim = 1.0 / np.sqrt(shp[0])
            out[name] = rng.uniform(-lim, lim, size=shp)
    return out


def flatten(params, layers=4):
    return np.concatenate([np.asarray(params[k], dtype=np.float64).ravel() for k in order(layers)])


def unflatten(flat, shapes, layers=4):
    out, o = {}, 0
    for k in order(layers):
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shapes[k])
        o += n
    return out


def _segments(seg):
    seg = np.asarray(seg)
    counts = np.diff(seg)
    inst = np.repeat(np.arange(len(counts)), counts)
    return inst, counts


def forward(params, x, seg, layers=4, quant=_ident):
    """Returns (y [R][d_out], cache) for features x [R][d_in] and instance offsets seg [B+1]."""
    inst, counts = _segments(seg)
    B = len(counts)
    h = x @ params["We"] + params["be"]
    cache = {"x": x, "inst": inst, "counts": counts, "h": [h], "z1": [], "a1": [], "pm": [], "quant": quant}
    for l in range(layers):
        z1 = quant(h) @ params[f"W1_{l}"] + params[f"b1_{l}"]
        a1 = np.maximum(z1, 0.0)
        pm = np.zeros((B, h.shape[1]))
        np.add.at(pm, inst, h)
        pm /= counts[:, None]
        q = quant(pm) @ params[f"Wp_{l}"]
        h = h + quant(a1) @ params[f"W2_{l}"] + params[f"b2_{l}"] + q[inst]
        cache["z1"].append(z1)
        cache["a1"].append(a1)
        cache["pm"].append(pm)
        cache["h"].append(h)
    y = quant(h) @ params["Wh"] + params["bh"]
    return y, cache


def loss(y, target, mask):
    """sum_r mask_r |y_r - t_r|^2 / (2 d_out sum_r mask_r) and dL/dy."""
    mask = np.asarray(mask, dtype=np.float64)
    cnt = y.shape[1] * mask.sum()
    diff = (y - target) * mask[:, None]
    return 0.5 * (diff * (y - target)).sum() / cnt, diff / cnt


def backward(params, cache, dy, layers=4):
    """Gradients of every parameter given dL/dy."""
    inst, counts, q = cache["inst"], cache["counts"], cache["quant"]
    B = len(counts)
    g = {}
    hL = cache["h"][layers]
    g["Wh"] = q(hL).T @ q(dy)
    g["bh"] = dy.sum(0)
    dh = q(dy) @ params["Wh"].T
    for l in range(layers - 1, -1, -1):
        h = cache["h"][l]
        a1, z1, pm = cache["a1"][l], cache["z1"][l], cache["pm"][l]
        # branch: relu(h W1 + b1) W2 + b2
        g[f"W2_{l}"] = q(a1).T @ q(dh)
        g[f"b2_{l}"] = dh.sum(0)
        da1 = q(dh) @ params[f"W2_{l}"].T
        dz1 = da1 * (z1 > 0)
        g[f"W1_{l}"] = q(h).T @ q(dz1)
        g[f"b1_{l}"] = dz1.sum(0)
        dh_branch = q(dz1) @ params[f"W1_{l}"].T
        # pool: mean_b(h) Wp broadcast to the instance's rows
        dq = np.zeros((B, dh.shape[1]))
        np.add.at(dq, inst, dh)
        g[f"Wp_{l}"] = q(pm).T @ q(dq)
        dpm = q(dq) @ params[f"Wp_{l}"].T
        dh_pool = (dpm / counts[:, None])[inst]
        dh = dh + dh_branch + dh_pool
    g["We"] = cache["x"].T @ dh
    g["be"] = dh.sum(0)
    return g


def adam(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place; state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k, gk in grads.items():
        m = state.setdefault("m_" + k, np.zeros_like(gk))
        v = state.setdefault("v_" + k, np.zeros_like(gk))
        m *= beta1
        m += (1 - beta1) * gk
        v *= beta2
        v += (1 - beta2) * gk * gk
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params
