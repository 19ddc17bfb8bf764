"""Learned proposal on the GPU: the BF16 MFMA product in its three forms,
forward and gradients against the FP64 oracle given the same BF16-rounded
weights, Adam training, and permutation equivariance.

The GPU rounds every operand of a product to BF16.  The oracle runs twice:
with the same BF16 rounding of the product operands (so ReLU gates are decided
at the kernel's operand precision) the bar per tensor is cosine >= 0.99999 and
a normwise relative error <= 5e-3 (what remains is FP32 versus FP64
accumulation and the odd operand landing on the other side of a BF16 rounding
midpoint); against the plain FP64 oracle, where ~0.2 % of ReLU gates flip and
the error norm grows like the square root of that share, cosine >= 0.998."""
import numpy as np
import pytest
import torch

from oracle import proposal as OP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "the GPU tests need a HIP device"
    from paper_2503_12204_amd import _lib
    return _lib


def _bf16(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16)


@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
@pytest.mark.parametrize("M,N,K", [(64, 64, 32), (70, 45, 37), (1, 200, 256), (256, 512, 1000), (33, 7, 5)])
def test_gemm_forms(L, ta, tb, M, N, K):
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.normal(size=(K, M) if ta else (M, K)).astype(np.float32)
    B = rng.normal(size=(N, K) if tb else (K, N)).astype(np.float32)
    Ab, Bb = _bf16(A), _bf16(B)
    C = L.gemm_bf16(Ab.cuda(), Bb.cuda(), M, N, K, ta, tb).cpu().numpy()
    a64 = Ab.float().numpy().astype(np.float64)
    b64 = Bb.float().numpy().astype(np.float64)
    ref = (a64.T if ta else a64) @ (b64.T if tb else b64)
    # FP32 accumulation of K exact BF16 products
    tol = 1e-5 * np.sqrt(K) * (np.abs(a64).max() * np.abs(b64).max() * np.sqrt(K)) + 1e-6
    assert np.abs(C - ref).max() <= tol
    # accumulate form
    C2 = L.gemm_bf16(Ab.cuda(), Bb.cuda(), M, N, K, ta, tb, C=torch.ones((M, N), device="cuda"), beta=1.0)
    assert np.abs(C2.cpu().numpy() - (ref + 1.0)).max() <= tol


@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
@pytest.mark.parametrize("M,N,K", [(2048, 2048, 96), (300, 200, 72), (129, 257, 8)])
def test_gemm_tiles_give_the_same_bits(L, ta, tb, M, N, K):
    """The 128x128 and 64x64 workgroup tiles accumulate every output element
    in the same order, so they give the same bits, ragged edges included
    (2048 x 2048 is where the default picks 128x128); the 128x128 result also
    meets the FP64 reference's bar."""
    rng = np.random.default_rng(M + N + K)
    A = rng.normal(size=(K, M) if ta else (M, K)).astype(np.float32)
    B = rng.normal(size=(N, K) if tb else (K, N)).astype(np.float32)
    Ab, Bb = _bf16(A).cuda(), _bf16(B).cuda()
    out = {}
    for tile in (64, 128):
        with L.option("gemm_tile", tile):
            out[tile] = L.gemm_bf16(Ab, Bb, M, N, K, ta, tb).cpu().numpy()
    assert np.array_equal(out[64], out[128])
    default = L.gemm_bf16(Ab, Bb, M, N, K, ta, tb).cpu().numpy()
    assert np.array_equal(default, out[64])
    a64 = Ab.cpu().float().numpy().astype(np.float64)
    b64 = Bb.cpu().float().numpy().astype(np.float64)
    ref = (a64.T if ta else a64) @ (b64.T if tb else b64)
    tol = 1e-5 * np.sqrt(K) * (np.abs(a64).max() * np.abs(b64).max() * np.sqrt(K)) + 1e-6
    assert np.abs(out[128] - ref).max() <= tol


def _problem(rng, R_per, d_in, d_out):
    seg = np.concatenate([[0], np.cumsum(R_per)]).astype(np.int32)
    R = int(seg[-1])
    x = rng.normal(size=(R, d_in)).astype(np.float32)
    t = rng.normal(size=(R, d_out)).astype(np.float32) * 0.5
    mask = (rng.uniform(size=R) > 0.2).astype(np.float32)
    mask[0] = 1.0
    return seg, x, t, mask


def _rounded(params):
    """Weights as the GPU uses them: matrices rounded to BF16, biases FP32."""
    out = {}
    for k, v in params.items():
        v32 = np.asarray(v, dtype=np.float32)
        out[k] = (_bf16(v32).float().numpy() if v.ndim == 2 else v32).astype(np.float64)
    return out


def _cos(a, b):
    return float((a * b).sum() / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


@pytest.mark.parametrize("shape", [dict(width=64, hidden=96, layers=2, d_out=20),
                                   dict(width=256, hidden=512, layers=4, d_out=200)])
def test_forward_and_gradients_match_oracle(L, shape):
    rng = np.random.default_rng(3)
    d_in = 6
    params = OP.init_params(rng, d_in, shape["width"], shape["hidden"], shape["layers"], shape["d_out"])
    for k in params:
        if params[k].ndim == 1:
            params[k] = rng.normal(size=params[k].shape) * 0.1
    seg, x, t, mask = _problem(rng, [3, 7, 1, 12, 5], d_in, shape["d_out"])
    net = L.ProposalNet(d_in=d_in, max_rows=64, max_batch=8, **shape)
    flat = OP.flatten(params, shape["layers"]).astype(np.float32)
    assert flat.size == net.n_params
    net.set_params(torch.as_tensor(flat, device="cuda"))
    xc, segc = torch.as_tensor(x, device="cuda"), torch.as_tensor(seg, device="cuda")
    y = net.forward(xc, segc).cpu().numpy()
    pr = _rounded(params)
    loss, g = net.gradients(xc, segc, torch.as_tensor(t, device="cuda"), torch.as_tensor(mask, device="cuda"))
    gg = OP.unflatten(g.cpu().numpy().astype(np.float64), OP.param_shapes(d_in, **{k: shape[k] for k in shape}),
                      shape["layers"])
    for quant, cos_bar, norm_bar in ((OP.bf16_round, 0.99999, 5e-3), (None, 0.998, None)):
        kw = {} if quant is None else {"quant": quant}
        yr, cache = OP.forward(pr, x.astype(np.float64), seg, shape["layers"], **kw)
        assert _cos(y.ravel(), yr.ravel()) >= cos_bar
        lr_, dy = OP.loss(yr, t.astype(np.float64), mask)
        assert abs(float(loss.cpu()) - lr_) <= 2e-2 * abs(lr_)
        gr = OP.backward(pr, cache, dy, shape["layers"])
        worst = []
        for name in OP.order(shape["layers"]):
            a, b = gg[name].ravel(), gr[name].ravel()
            worst.append((name, _cos(a, b), np.linalg.norm(a - b) / np.linalg.norm(b)))
        print("quantised" if quant else "fp64", min(worst, key=lambda w: w[1]), max(worst, key=lambda w: w[2]))
        for name, c, nr in worst:
            assert c >= cos_bar, (name, c)
            if norm_bar is not None:
                assert nr <= norm_bar, (name, nr)
    net.close()


def test_training_reduces_loss_and_stays_equivariant(L):
    rng = np.random.default_rng(5)
    d_in, d_out = 6, 20
    seg, x, _, _ = _problem(rng, [4, 6, 5, 9, 8, 4], d_in, d_out)
    proj = rng.normal(size=(d_in, d_out)) * 0.3
    t = np.tanh(x @ proj).astype(np.float32)          # a smooth per-robot target
    mask = np.ones(x.shape[0], dtype=np.float32)
    net = L.ProposalNet(d_in=d_in, width=64, hidden=128, layers=2, d_out=d_out, max_rows=64, max_batch=8, seed=1)
    xc, segc = torch.as_tensor(x, device="cuda"), torch.as_tensor(seg, device="cuda")
    tc, mc = torch.as_tensor(t, device="cuda"), torch.as_tensor(mask, device="cuda")
    first = float(net.train_step(xc, segc, tc, mc, 3e-3).cpu())
    for _ in range(300):
        last = net.train_step(xc, segc, tc, mc, 3e-3)
    last = float(last.cpu())
    assert last < 0.1 * first, (first, last)
    # permuting the robots of each instance permutes the predictions
    perm = np.concatenate([seg[i] + rng.permutation(seg[i + 1] - seg[i]) for i in range(len(seg) - 1)])
    y = net.forward(xc, segc).cpu().numpy()
    yp = net.forward(torch.as_tensor(x[perm], device="cuda"), segc).cpu().numpy()
    assert np.allclose(yp, y[perm], rtol=0, atol=1e-4 * np.abs(y).max())
    net.close()


def test_adam_step_matches_oracle(L):
    rng = np.random.default_rng(7)
    shape = dict(width=32, hidden=48, layers=1, d_out=10)
    params = OP.init_params(rng, 6, **shape)
    seg, x, t, mask = _problem(rng, [5, 3], 6, 10)
    net = L.ProposalNet(d_in=6, max_rows=16, max_batch=4, **shape)
    flat = OP.flatten(params, 1).astype(np.float32)
    net.set_params(torch.as_tensor(flat, device="cuda"))
    xc, segc = torch.as_tensor(x, device="cuda"), torch.as_tensor(seg, device="cuda")
    _, g = net.gradients(xc, segc, torch.as_tensor(t, device="cuda"), torch.as_tensor(mask, device="cuda"))
    net.train_step(xc, segc, torch.as_tensor(t, device="cuda"), torch.as_tensor(mask, device="cuda"), 1e-2)
    w1 = net.get_params().cpu().numpy().astype(np.float64)
    gd = g.cpu().numpy().astype(np.float64)
    # first Adam step from zero moments: w - lr g / (|g| + eps), with the GPU's own gradient
    expect = flat.astype(np.float64) - 1e-2 * gd / (np.abs(gd) + 1e-8)
    assert np.abs(w1 - expect).max() <= 1e-6
    net.close()
