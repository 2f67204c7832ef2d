"""Warm-start network: an addition to the method, not part of the paper.

Test infrastructure: a plain FP64 reference of the network that predicts the
start coefficients alpha_0 from the measured fields.  Only tests, the smoke
check and the benchmark's CPU baseline use it.

Network: four affine layers with exact GELU between them,
    h_0 = s_in * x,  z_l = h_{l-1} W_l^T + b_l,  h_l = gelu(z_l)  (l < L),
    y = z_L,
with W_l of shape [n_out, n_in] (row per output unit).  x is the measured
field E_sca [Ni][Ns] as interleaved (Re, Im) reals; y is alpha_0 [Ni][K][K]
as interleaved (Re, Im) reals divided by s_out.  The loss is the mean squared
error over all outputs of the batch.  gelu(z) = z Phi(z) with the standard
normal distribution function Phi.

With quant=True the GEMM operands are rounded to bfloat16 (round to nearest,
ties to even) where the device rounds them: the layer input h_{l-1} and the
weights in the forward pass, the gradient dz_l and the weights / stored
activations in the backward pass.  Sums, biases, GELU and the loss stay in
FP64 here.  Pins: the FP64 network against torch float64 autograd and
central differences, the rounding against torch's bfloat16 conversion, Adam
against torch.optim.Adam; where the rounding points sit follows the device
design (the paper has no such network).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _q(a, quant):
    return bf16_round(a) if quant else np.asarray(a, dtype=np.float64)


def forward(params, x, s_in=1.0, quant=False):
    """params: list of (W [n_out, n_in], b [n_out]).  Returns y and the cache for backward."""
    h = s_in * np.asarray(x, dtype=np.float64)
    cache = []
    L = len(params)
    for l, (W, b) in enumerate(params):
        a = _q(h, quant)
        z = a @ _q(W, quant).T + b
        cache.append((a, z))
        h = gelu(z) if l < L - 1 else z
    return h, cache


def mse(y, t):
    """Mean squared error over every output of the batch and its derivative in y."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, cache, dy, quant=False):
    """Gradients [(dW_l, db_l)] of a scalar whose derivative in y is dy."""
    grads = [None] * len(params)
    dz = np.asarray(dy, dtype=np.float64)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        a, _z = cache[l]
        dzq = _q(dz, quant)
        grads[l] = (dzq.T @ a, dz.sum(axis=0))
        if l > 0:
            dh = dzq @ _q(W, quant)
            dz = dh * gelu_grad(cache[l - 1][1])
    return grads


def adam_update(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Bias-corrected Adam on a real array; t counts steps from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    step = lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)
    return w - step, m, v


def train_step(params, state, x, t_target, t, lr, s_in=1.0, quant=False):
    """One MSE step: forward, backward, Adam on every weight and bias.  state: [(mW, vW, mb, vb)]."""
    y, cache = forward(params, x, s_in, quant)
    loss, dy = mse(y, t_target)
    grads = backward(params, cache, dy, quant)
    new_p, new_s = [], []
    for (W, b), (gW, gb), (mW, vW, mb, vb) in zip(params, grads, state):
        W2, mW, vW = adam_update(W, gW, mW, vW, t, lr)
        b2_, mb, vb = adam_update(b, gb, mb, vb, t, lr)
        new_p.append((W2, b2_))
        new_s.append((mW, vW, mb, vb))
    return new_p, new_s, loss
