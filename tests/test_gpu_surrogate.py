"""GPU coarse-stepper network against the surrogate oracle.

Layer checks use the GPU's own stored BF16 inputs of each layer, so the comparison isolates one
kernel: a BF16 output may differ from the FP64 oracle's only where the FP32 accumulation lands on
the other side of a rounding boundary (at most one BF16 ulp, on a small fraction of values)."""
import numpy as np
import pytest
import torch

from oracle import surrogate as S
from paper_2507_21748_amd.inputs import quench_field, surrogate_init

pytestmark = pytest.mark.gpu


def _params(seed=3):
    th = surrogate_init(seed).astype(np.float64)
    th += np.random.default_rng(seed).normal(0, 0.02, th.shape)  # non-zero biases
    return th.astype(np.float32)


def _bf(t):
    return t.float().cpu().numpy().astype(np.float64)


def _rounded_close(got, exact, absum, frac=2e-3):
    """got = bf16 of an FP32 evaluation of `exact` (FP64): |FP32 - FP64| <= 2e-6 sum|terms| (a
    bound on FP32 accumulation over <= 864 terms), plus at most half a BF16 ulp (2^-8 relative)
    for the final rounding; and at most `frac` of the values differ from bf16(exact)."""
    got = np.asarray(got, np.float64)
    exact = np.asarray(exact, np.float64)
    e = 2e-6 * np.asarray(absum, np.float64)
    bound = 2.0 ** -8 * (np.abs(exact) + e) + e + 1e-38
    assert np.all(np.abs(got - exact) <= bound), np.max(np.abs(got - exact) / bound)
    assert np.mean(got != S.bf16(exact)) <= frac, np.mean(got != S.bf16(exact))


@pytest.mark.parametrize("n", [24, 21])
def test_train_step_layers_match_oracle(evx_gpu, n):
    """n = 21 leaves ragged weight-gradient tiles along x (8-voxel rows) and y (16 rows)."""
    from paper_2507_21748_amd.surrogate import Net
    halo = 4
    theta = _params()
    net = Net(theta)
    c = quench_field((n, n, n), 0.1, 0.6, seed=21)
    t = quench_field((n, n, n), 0.1, 0.6, seed=22)
    x = torch.from_numpy(c).cuda()[None].contiguous()
    y = torch.from_numpy(t).cuda()[None].contiguous()
    loss = net.train_step(x, y, halo, lr=1e-30).item()
    torch.cuda.synchronize()
    b = net.train_buffers(n)
    P = S.unpack(theta)
    x0 = _bf(b["x0"])
    assert np.array_equal(x0, S.bf16(c))
    inp = x0[..., None]
    for li, (zk, ak) in enumerate((("z1", "a1"), ("z2", "a2"), ("z3", "a3"))):
        W, bias = P[li]
        acc = S.conv3d(inp, S.bf16(W), bias)
        absum = S.conv3d(np.abs(inp), np.abs(S.bf16(W)), np.abs(bias))
        z_gpu = _bf(b[zk])
        _rounded_close(z_gpu, acc, absum)
        g_exact = S.gelu(z_gpu)
        _rounded_close(_bf(b[ak]), g_exact, np.abs(g_exact))
        inp = _bf(b[ak])
    W4, b4 = P[3]
    out_ref = c.astype(np.float64) + S.conv3d(inp, S.bf16(W4), b4)[..., 0]
    out = b["out"].cpu().numpy().astype(np.float64)
    assert np.linalg.norm(out - out_ref) / np.linalg.norm(out_ref) <= 1e-6
    inner = (n - 2 * halo) ** 3
    d = np.zeros_like(out)
    sl = slice(halo, n - halo)
    d[sl, sl, sl] = (out - t)[sl, sl, sl]
    assert abs(loss / (np.sum(d * d) / inner) - 1) <= 1e-5
    dy_ref = 2.0 / inner * d
    dy = b["dy"].cpu().numpy()
    assert np.max(np.abs(dy - dy_ref)) <= 1e-6 * np.max(np.abs(dy_ref))
    # backward on the GPU's stored activations
    acts = [x0[..., None], _bf(b["a1"]), _bf(b["a2"]), _bf(b["a3"])]
    pres = [_bf(b["z1"]), _bf(b["z2"]), _bf(b["z3"])]
    g = dy[..., None].astype(np.float64)
    grads = []
    gpu_dz = {3: _bf(b["dz3"]), 2: _bf(b["dz2"]), 1: _bf(b["dz1"])}
    for li in range(3, -1, -1):
        gW = S.conv3d_weight_grad(g, acts[li])
        gb = g.reshape(-1, g.shape[-1]).sum(axis=0)
        grads.append((li, gW, gb))
        if li > 0:
            Wb = S.bf16(P[li][0])
            gp = S.gelu_prime(pres[li - 1])
            exact = S.conv3d_transpose(g, Wb) * gp
            absum = S.conv3d_transpose(np.abs(g), np.abs(Wb)) * np.abs(gp)
            g = S.bf16(exact)
            _rounded_close(gpu_dz[li], exact, absum, frac=5e-3)
            g = gpu_dz[li]                # continue from the GPU's own rounding
    gflat = b["grads"].cpu().numpy().astype(np.float64)
    off = 0
    offs = []
    for (wshape, bshape) in S.layer_shapes():
        offs.append(off)
        off += int(np.prod(wshape)) + bshape[0]
    for li, gW, gb in grads:
        nw = gW.size
        got_w = gflat[offs[li]:offs[li] + nw].reshape(gW.shape)
        got_b = gflat[offs[li] + nw:offs[li] + nw + gb.size]
        assert np.linalg.norm(got_w - gW) <= 1e-4 * np.linalg.norm(gW), li
        assert np.linalg.norm(got_b - gb) <= 1e-4 * np.linalg.norm(gb) + 1e-12, li


def test_adam_update_matches_oracle(evx_gpu):
    """Three training steps at a real learning rate: each step's parameters and Adam moments on
    the GPU equal the oracle's Adam update (Kingma & Ba, with bias correction) applied in FP64 to
    the GPU's own parameters, moments and summed gradient before that step, to FP32 rounding."""
    from paper_2507_21748_amd.surrogate import Net
    n, halo, lr = 20, 4, 3e-3
    net = Net(_params(5))
    x = torch.from_numpy(quench_field((n, n, n), 0.0, 0.6, seed=51)).cuda()[None].contiguous()
    y = torch.from_numpy(quench_field((n, n, n), 0.0, 0.6, seed=52)).cuda()[None].contiguous()

    def close(got, ref, scale):
        """FP32 evaluation of a few terms whose magnitudes sum to `scale`: within 1e-6 of it
        (a handful of FP32 roundings, 6e-8 each), so a cancelling sum is not held to a
        relative bound on its small result."""
        got = got.cpu().numpy().astype(np.float64)
        tol = 1e-6 * scale + 1e-30
        assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)

    for step in range(1, 4):
        th0 = net.params.cpu().numpy().astype(np.float64)
        m0 = net.m.cpu().numpy().astype(np.float64)
        v0 = net.v.cpu().numpy().astype(np.float64)
        net.train_step(x, y, halo, lr=lr)
        torch.cuda.synchronize()
        assert net.step == step
        g = net.train_buffers(n)["grads"].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(g) > 0
        th_ref, m_ref, v_ref = S.adam_update(th0, m0, v0, g, step, lr)
        close(net.m, m_ref, 0.9 * np.abs(m0) + 0.1 * np.abs(g))
        close(net.v, v_ref, 0.999 * v0 + 0.001 * g * g)
        close(net.params, th_ref, np.abs(th0) + np.abs(th_ref - th0))
        # the update moved the parameters by about lr per element (Adam's normalised step)
        moved = np.abs(th_ref - th0)
        assert np.median(moved) > 0.1 * lr


def test_gelu_over_wide_preactivations(evx_gpu):
    """First-layer weights scaled up so that its BF16 pre-activations reach past +-8 and down to
    below 2^-8 in magnitude: the stored activations equal bf16(GELU(z)) of the FP64 oracle on every
    range the GPU evaluates differently (table, small-argument series, large-argument paths)."""
    from paper_2507_21748_amd.surrogate import Net
    theta = _params(9).astype(np.float64)
    (w_shape, b_shape) = S.layer_shapes()[0]
    nw = int(np.prod(w_shape)) + b_shape[0]
    theta[:nw] *= 4.0  # z in about [-11.4, 11.9]: no FP32 denormal results
    net = Net(theta.astype(np.float32))
    n = 24
    c = torch.from_numpy(quench_field((n, n, n), 0.0, 0.8, seed=26)).cuda()[None].contiguous()
    net.train_step(c, c, 4, lr=1e-30)
    torch.cuda.synchronize()
    b = net.train_buffers(n)
    z = _bf(b["z1"])
    a = _bf(b["a1"])
    assert (z >= 8).any() and (z <= -8).any() and ((np.abs(z) < 2.0 ** -8) & (z != 0)).any()
    exact = S.gelu(z)
    _rounded_close(a, exact, np.abs(exact))


def test_infer_equals_training_forward(evx_gpu):
    from paper_2507_21748_amd.surrogate import Net
    n = 24
    net = Net(_params())
    c = torch.from_numpy(quench_field((n, n, n), 0.1, 0.6, seed=21)).cuda()
    net.train_step(c[None].contiguous(), c[None].contiguous(), 4, lr=1e-30)
    ref = net.train_buffers(n)["out"].clone()
    net.set_params(net.params)
    out = net.infer(c)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


@pytest.mark.parametrize("shape", [(16, 24, 32), (20, 12, 40), (9, 10, 18), (1, 8, 40), (2, 20, 6)])
def test_infer_matches_oracle(evx_gpu, shape):
    """Full network on grids with partial MFMA tiles: the prediction net(c) within 5e-3 relative
    L2 of the FP64 oracle (BF16 rounding flips propagate through three layers). The last two
    grids are one and two planes deep and narrower than a halo, so halo points wrap onto the
    same planes and columns several times."""
    from paper_2507_21748_amd.surrogate import Net
    theta = _params(4)
    net = Net(theta)
    c = quench_field(shape, 0.0, 0.6, seed=23)
    out = net.infer(torch.from_numpy(c).cuda()).cpu().numpy().astype(np.float64)
    ref = S.forward(c, theta)
    dy = out - c
    dy_ref = ref - c
    assert np.linalg.norm(dy - dy_ref) / np.linalg.norm(dy_ref) <= 5e-3


def test_translation_equivariance_on_gpu(evx_gpu):
    from paper_2507_21748_amd.surrogate import Net
    net = Net(_params(5))
    c = torch.from_numpy(quench_field((32, 32, 48), 0.0, 0.5, seed=24)).cuda()
    a = net.infer(torch.roll(c, (4, 8, 16), (0, 1, 2)).contiguous())
    b = torch.roll(net.infer(c), (4, 8, 16), (0, 1, 2))
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_training_on_solver_pairs_reduces_loss(evx_gpu):
    from paper_2507_21748_amd import evx
    from paper_2507_21748_amd.surrogate import Net, make_pairs, sample_windows
    prm = evx.CHParams(dt=0.5)
    pairs = make_pairs((64, 64, 64), [0.0, 0.2], [101], 200, 10, 10, prm)
    rng = np.random.default_rng(0)
    net = Net(seed=7)
    first = last = None
    for it in range(150):
        x, y = sample_windows(pairs, 4, 40, rng)
        L = net.train_step(x, y, 4, lr=1e-3).item()
        first = L if first is None else first
        last = L
    print(f"surrogate training loss {first:.3e} -> {last:.3e}")
    assert last < 0.5 * first


def test_mass_projection(evx_gpu):
    """With mass conservation on, the prediction's mean equals the input's (FP64 sum check) and
    the increment differs from the plain one by a constant."""
    from paper_2507_21748_amd.surrogate import Net
    net = Net(_params(6))
    c = torch.from_numpy(quench_field((32, 40, 48), 0.2, 0.3, seed=25)).cuda()
    plain = net.infer(c)
    cons = net.infer(c, conserve_mass=True)
    torch.cuda.synchronize()
    d = (cons.double() - plain.double())
    assert abs(float(cons.double().mean() - c.double().mean())) <= 1e-7
    assert float(d.max() - d.min()) <= 1e-6


def test_infer_512_sampled_voxels(evx_gpu):
    """The full-size inference (512^3, the rollout grid) against the FP64 oracle on sampled voxels:
    an output voxel depends only on the input within distance 4 (four 3x3x3 layers), so the
    oracle's network on the periodic 9^3 neighbourhood gives that voxel exactly."""
    from paper_2507_21748_amd.surrogate import Net
    n = 512
    theta = _params(8)
    net = Net(theta)
    c_np = quench_field((n, n, n), 0.0, 0.05, seed=7)
    out = net.infer(torch.from_numpy(c_np).cuda()).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(9)
    pts = rng.integers(0, n, size=(24, 3))
    pts[0] = (0, 0, 0)              # periodic wrap on every axis
    pts[1] = (n - 1, n - 1, n - 1)
    got, ref, base = [], [], []
    r = np.arange(-4, 5)
    for z, y, x in pts:
        patch = c_np[np.ix_((z + r) % n, (y + r) % n, (x + r) % n)]
        ref.append(S.forward(patch, theta)[4, 4, 4])
        got.append(out[z, y, x])
        base.append(float(c_np[z, y, x]))
    got, ref, base = map(np.asarray, (got, ref, base))
    assert np.linalg.norm((got - base) - (ref - base)) <= 1e-2 * np.linalg.norm(ref - base)
