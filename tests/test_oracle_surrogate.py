"""Pins of the surrogate oracle (no GPU): its convolution, transpose and weight gradient against
torch's float64 conv3d with circular padding and autograd, its BF16 rounding against torch's
bfloat16 cast, its full backward against torch autograd with rounding switched off, translation
equivariance, and its Adam step against torch.optim.Adam."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import surrogate as S
from paper_2507_21748_amd.inputs import quench_field, surrogate_init


def _torch_w(W):
    co, ci = W.shape[1], W.shape[2]
    return torch.from_numpy(W.reshape(3, 3, 3, co, ci).transpose(3, 4, 0, 1, 2).copy())


def _torch_conv(x, W, b=None):
    xt = torch.from_numpy(np.moveaxis(x, -1, 0)[None].copy())
    xp = F.pad(xt, (1, 1, 1, 1, 1, 1), mode="circular")
    y = F.conv3d(xp, _torch_w(W), None if b is None else torch.from_numpy(b))
    return np.moveaxis(y[0].numpy(), 0, -1)


@pytest.mark.parametrize("ci,co", [(1, 32), (32, 32), (32, 1), (3, 5)])
def test_conv3d_matches_torch_circular(ci, co):
    rng = np.random.default_rng(ci * 100 + co)
    x = rng.standard_normal((5, 6, 7, ci))
    W = rng.standard_normal((27, co, ci))
    b = rng.standard_normal(co)
    assert np.allclose(S.conv3d(x, W, b), _torch_conv(x, W, b), atol=1e-12, rtol=1e-12)


def test_transpose_and_weight_grad_match_torch_autograd():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 5, 6, 3))
    W = rng.standard_normal((27, 4, 3))
    g = rng.standard_normal((4, 5, 6, 4))
    xt = torch.from_numpy(np.moveaxis(x, -1, 0)[None].copy()).requires_grad_(True)
    wt = _torch_w(W).requires_grad_(True)
    y = F.conv3d(F.pad(xt, (1, 1, 1, 1, 1, 1), mode="circular"), wt)
    y.backward(torch.from_numpy(np.moveaxis(g, -1, 0)[None].copy()))
    gx = np.moveaxis(xt.grad[0].numpy(), 0, -1)
    gw = wt.grad.numpy().transpose(2, 3, 4, 0, 1).reshape(27, 4, 3)
    assert np.allclose(S.conv3d_transpose(g, W), gx, atol=1e-11)
    assert np.allclose(S.conv3d_weight_grad(g, x), gw, atol=1e-11)


def test_bf16_matches_torch():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(10000) * 10 ** rng.uniform(-6, 6, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(x), ref)


def test_gelu_prime_is_derivative():
    z = np.linspace(-6, 6, 241)
    h = 1e-6
    fd = (S.gelu(z + h) - S.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - S.gelu_prime(z))) < 1e-8
    assert np.allclose(S.gelu(z), torch.nn.functional.gelu(torch.from_numpy(z)).numpy(),
                       atol=1e-15)


def test_translation_equivariance():
    theta = surrogate_init(1)
    c = quench_field((6, 8, 10), 0.0, 0.5, seed=2)
    a = S.forward(np.roll(c, (1, 2, 3), axis=(0, 1, 2)), theta)
    b = np.roll(S.forward(c, theta), (1, 2, 3), axis=(0, 1, 2))
    assert np.array_equal(a, b)


def test_loss_gradient_matches_torch_without_rounding(monkeypatch):
    """With BF16 rounding switched off the oracle's loss and gradient equal torch autograd of the
    same network in float64 (pins every term of the backward pass)."""
    monkeypatch.setattr(S, "bf16", lambda x: np.asarray(x, dtype=np.float64))
    theta = surrogate_init(5).astype(np.float64) * 1.0
    theta += np.random.default_rng(6).normal(0, 0.01, theta.shape)   # non-zero biases too
    cs = [quench_field((8, 8, 8), 0.1, 0.5, seed=s).astype(np.float64) for s in (7, 8)]
    ts = [quench_field((8, 8, 8), 0.1, 0.5, seed=s).astype(np.float64) for s in (9, 10)]
    L, g = S.loss_and_grads(cs, ts, theta, halo=2)

    th = torch.from_numpy(theta.copy()).requires_grad_(True)
    k = 0
    params = []
    for (ci, co) in S.LAYERS:
        nw = 27 * co * ci
        W = th[k:k + nw].reshape(3, 3, 3, co, ci).permute(3, 4, 0, 1, 2)
        params.append((W, th[k + nw:k + nw + co]))
        k += nw + co
    tot, n = 0.0, 0
    for c, t in zip(cs, ts):
        x = torch.from_numpy(c)[None, None]
        h = x
        for li, (W, b) in enumerate(params):
            h = F.conv3d(F.pad(h, (1, 1, 1, 1, 1, 1), mode="circular"), W, b)
            if li < 3:
                h = F.gelu(h)
        d = (x + h - torch.from_numpy(t)[None, None])[..., 2:6, 2:6, 2:6]
        tot = tot + (d * d).sum()
        n += d.numel()
    (tot / n).backward()
    assert abs(L - float(tot.detach() / n)) < 1e-12 * max(1.0, L)
    assert np.allclose(g, th.grad.numpy(), atol=1e-12, rtol=1e-9)


def test_adam_matches_torch():
    rng = np.random.default_rng(11)
    p0 = rng.standard_normal(50)
    gs = [rng.standard_normal(50) for _ in range(5)]
    pt = torch.from_numpy(p0.copy()).requires_grad_(True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for i, g in enumerate(gs):
        opt.zero_grad()
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = S.adam_update(p, m, v, g, i + 1, 1e-3)
    assert np.allclose(p, pt.detach().numpy(), atol=1e-14)


def test_param_count():
    assert S.param_count() == 57121 == surrogate_init(0).size
