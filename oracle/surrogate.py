"""FP64 CPU oracle for the learned coarse stepper: a periodic 3D residual CNN
c_out = c + net(c), net = conv4(gelu(conv3(gelu(conv2(gelu(conv1(c))))))), 3x3x3 kernels,
channels 1 -> 32 -> 32 -> 32 -> 1, trained with Adam on solver trajectories.

TEST INFRASTRUCTURE ONLY (see oracle/ch.py).  The paper motivates neural-surrogate training on
solver data and backpropagation through voxel solvers (Statement of Need); the network itself is
this build's specification:

  * conv(x)[v, o] = b[o] + sum_i sum_{d in {-1,0,1}^3} W[d, o, i] x[(v + d) mod grid, i]
    (cross-correlation with circular padding, as torch.nn.functional.conv3d); weights are stored
    as W[27, Cout, Cin] with d = (dz, dy, dx) -> 9 (dz+1) + 3 (dy+1) + (dx+1);
  * gelu(z) = z Phi(z) (exact erf form), gelu'(z) = Phi(z) + z phi(z);
  * BF16 storage, FP32 (here FP64) accumulation: the network input bf16(c), the weights, every
    pre-activation zb = bf16(conv + b), every activation bf16(gelu(zb)) are rounded to bfloat16
    (round to nearest even); the last layer's output and the residual add stay in float;
  * loss = mean over the window interior of (c + net(c) - target)^2;
  * Adam (Kingma & Ba) on FP32 master weights: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Backward (per layer, gz = dL/dz): dW[d, o, i] = sum_v gz[v, o] x[v + d, i], db = sum_v gz,
dx[v, i] = sum_d sum_o W[d, o, i] gz[v - d, o], and gz_prev = dx * gelu'(zb_prev), with the
same BF16 rounding of gz_prev that the GPU applies before its next product.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["bf16", "layer_shapes", "param_count", "unpack", "conv3d", "gelu", "gelu_prime",
           "forward", "loss_and_grads", "adam_update", "OFFSETS"]

CH = 32
LAYERS = [(1, CH), (CH, CH), (CH, CH), (CH, 1)]
OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16(x):
    """Round float values to bfloat16 (nearest, ties to even) and return them as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


def layer_shapes():
    return [((27, co, ci), (co,)) for ci, co in LAYERS]


def param_count() -> int:
    return sum(27 * co * ci + co for ci, co in LAYERS)


def unpack(theta):
    """Flat FP32 parameter vector -> [(W[27, Cout, Cin], b[Cout])] (layer order)."""
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for (wshape, bshape) in layer_shapes():
        nw = int(np.prod(wshape))
        out.append((theta[k:k + nw].reshape(wshape), theta[k + nw:k + nw + bshape[0]]))
        k += nw + bshape[0]
    return out


def conv3d(x, W, b=None):
    """x [nz, ny, nx, Cin] -> [nz, ny, nx, Cout], circular cross-correlation, FP64."""
    y = np.zeros(x.shape[:3] + (W.shape[1],))
    for d, (dz, dy, dx) in enumerate(OFFSETS):
        xs = np.roll(x, shift=(-dz, -dy, -dx), axis=(0, 1, 2))  # xs[v] = x[v + d]
        y += xs @ W[d].T
    if b is not None:
        y += b
    return y


def conv3d_transpose(g, W):
    """dx[v, i] = sum_d sum_o W[d, o, i] g[v - d, o]."""
    out = np.zeros(g.shape[:3] + (W.shape[2],))
    for d, (dz, dy, dx) in enumerate(OFFSETS):
        gs = np.roll(g, shift=(dz, dy, dx), axis=(0, 1, 2))  # gs[v] = g[v - d]
        out += gs @ W[d]
    return out


def conv3d_weight_grad(g, x):
    """dW[d, o, i] = sum_v g[v, o] x[v + d, i]."""
    co, ci = g.shape[-1], x.shape[-1]
    dW = np.zeros((27, co, ci))
    g2 = g.reshape(-1, co)
    for d, (dz, dy, dx) in enumerate(OFFSETS):
        xs = np.roll(x, shift=(-dz, -dy, -dx), axis=(0, 1, 2)).reshape(-1, ci)
        dW[d] = g2.T @ xs
    return dW


def _Phi(z):
    """Standard normal CDF via erfc, accurate also in the far negative tail (1 + erf would
    cancel there)."""
    return 0.5 * np.vectorize(math.erfc)(-z / math.sqrt(2.0))


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return z * _Phi(z)


def gelu_prime(z):
    z = np.asarray(z, dtype=np.float64)
    Phi = _Phi(z)
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return Phi + z * phi


def forward(c, theta, keep=False):
    """c [nz, ny, nx] float -> c + net(c).  With keep, also returns the stored activations
    (inputs of each layer, BF16 values) and pre-activations (BF16 values)."""
    params = unpack(theta)
    x = bf16(np.asarray(c, dtype=np.float64))[..., None]
    inputs, pre = [], []
    for li, (W, b) in enumerate(params):
        Wb = bf16(W)
        inputs.append(x)
        acc = conv3d(x, Wb, b)
        if li < len(params) - 1:
            zb = bf16(acc)
            pre.append(zb)
            x = bf16(gelu(zb))
        else:
            y = acc[..., 0]
    out = np.asarray(c, dtype=np.float64) + y
    return (out, inputs, pre) if keep else out


def loss_and_grads(cs, targets, theta, halo):
    """Mean squared error over the interiors (halo cut from every face) of a batch of windows and
    its gradient w.r.t. the flat parameter vector (FP64)."""
    params = unpack(theta)
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    n_int = 0
    loss = 0.0
    diffs = []
    for c, t in zip(cs, targets):
        out, inputs, pre = forward(c, theta, keep=True)
        mask = np.zeros(c.shape, dtype=bool)
        mask[halo:c.shape[0] - halo, halo:c.shape[1] - halo, halo:c.shape[2] - halo] = True
        d = np.where(mask, out - np.asarray(t, dtype=np.float64), 0.0)
        diffs.append((d, inputs, pre))
        loss += float(np.sum(d * d))
        n_int += int(mask.sum())
    loss /= n_int
    for d, inputs, pre in diffs:
        g = (2.0 / n_int) * d[..., None]
        for li in range(len(params) - 1, -1, -1):
            W, _ = params[li]
            Wb = bf16(W)
            gW, gb = grads[li]
            gW += conv3d_weight_grad(g, inputs[li])
            gb += g.reshape(-1, g.shape[-1]).sum(axis=0)
            if li > 0:
                gx = conv3d_transpose(g, Wb)
                g = bf16(gx * gelu_prime(pre[li - 1]))
    flat = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])
    return loss, flat


def adam_update(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
