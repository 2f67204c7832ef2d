"""Untrained FCNN reparameterisation of the Fourier coefficients (Sec. 3.1, Fig. 4).

TEST INFRASTRUCTURE ONLY: plain FP64 NumPy, imported by tests/, the smoke check
and the CPU baseline of the benchmark, never by the product path.

The solver of Sec. 3.1 does not optimise the coefficients directly: an FCNN
whose input is the real and imaginary parts of the start coefficients alpha_0
predicts a correction, alpha_hat = alpha_0 + Delta alpha, and Adam (Sec. 3.3)
trains the network's weights on the composite loss (Eq. 13) at alpha_hat.

The paper gives the layer sizes only in a figure that is not available, so
this module fixes them (a reading, not the paper's numbers):
  * one network per reconstruction, shared by its N_i incidences: each
    incidence is one input row [Re alpha_0[i, :], Im alpha_0[i, :]] of width
    D = 2 K^2 (the two channels, flattened mode by mode in the K x K order of
    the coefficients), and one output row [Re, Im] of Delta alpha[i, :];
  * three dense layers D -> H -> H -> D, tanh after the first two;
  * two scalars set the scales: the input rows are s_in [Re, Im] alpha_0 and
    Delta alpha = s_out times the output rows.  With s_in = 1 / rms(alpha_0)
    (unit-scale inputs) and s_out = 1 / H, the first Adam step moves
    alpha_hat by about as much as a direct Adam step moves alpha at the same
    learning rate; s_in = s_out = 1 is the plain network;
  * parameters of one reconstruction, flat and in this order: for each layer
    a block of (in + 1) x out numbers, row-major [k][n]; rows 0..in-1 hold
    the weights (z[n] = sum_k x[k] W[k][n] + W[in][n]), row `in` the bias.

Gradient convention: g = dL/dRe + i dL/dIm of alpha_hat (as the loss module
returns it), so the output layer's upstream gradient is [Re g, Im g].
"""
from __future__ import annotations

import numpy as np

from . import loss as _loss
from . import mlp as _mlp


def layer_shapes(K: int, H: int):
    D = 2 * K * K
    return [(D, H), (H, H), (H, D)]


def n_params(K: int, H: int) -> int:
    return sum((i + 1) * o for i, o in layer_shapes(K, H))


def unpack(theta_b: np.ndarray, K: int, H: int):
    """Views (W [in][out], bias [out]) of one reconstruction's flat parameters."""
    out, off = [], 0
    for i, o in layer_shapes(K, H):
        blk = theta_b[off:off + (i + 1) * o].reshape(i + 1, o)
        out.append((blk[:i], blk[i]))
        off += (i + 1) * o
    return out


def split(z: np.ndarray) -> np.ndarray:
    """[N_i][K][K] complex -> [N_i][2 K^2] real rows (Re block, then Im block)."""
    z = z.reshape(z.shape[0], -1)
    return np.concatenate([z.real, z.imag], axis=1)


def join(y: np.ndarray, K: int) -> np.ndarray:
    q = K * K
    return (y[:, :q] + 1j * y[:, q:]).reshape(y.shape[0], K, K)


def forward(theta_b: np.ndarray, alpha0_b: np.ndarray, K: int, H: int, s_in: float = 1.0, s_out: float = 1.0):
    """alpha_hat of one reconstruction and the activations the gradient needs."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta_b, K, H)
    X = split(s_in * alpha0_b)
    A1 = np.tanh(X @ W1 + b1)
    A2 = np.tanh(A1 @ W2 + b2)
    Y = A2 @ W3 + b3
    return alpha0_b + s_out * join(Y, K), (X, A1, A2)


def backward(theta_b: np.ndarray, cache, g_b: np.ndarray, K: int, H: int, s_out: float = 1.0) -> np.ndarray:
    """Flat gradient of L with respect to theta_b, given g = dL/dRe + i dL/dIm of alpha_hat
    (the chain rule through alpha_hat = alpha_0 + s_out join(Y))."""
    (W1, _), (W2, _), (W3, _) = unpack(theta_b, K, H)
    X, A1, A2 = cache
    G3 = s_out * split(g_b)              # dL/dY
    G2 = (G3 @ W3.T) * (1.0 - A2 * A2)   # dL/dZ2
    G1 = (G2 @ W2.T) * (1.0 - A1 * A1)   # dL/dZ1
    parts = []
    for inp, G in ((X, G1), (A1, G2), (A2, G3)):
        parts.append(np.vstack([inp.T @ G, G.sum(axis=0)[None, :]]).ravel())
    return np.concatenate(parts)


def step(theta_b, m_b, v_b, t: int, alpha0_b, prob: _loss.Problem, K: int, H: int, lr: float = 1e-2,
         b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, s_in: float = 1.0, s_out: float = 1.0):
    """One Adam step (Sec. 3.3) on the weights of one reconstruction.

    theta_b, m_b, v_b: [n_params]; alpha0_b: [N_i][K][K]; t counts steps from 1.
    Returns the updated (theta, m, v), alpha_hat at the weights before the
    update, and the loss module's record at that alpha_hat."""
    alpha_hat, cache = forward(theta_b, alpha0_b, K, H, s_in, s_out)
    out = _loss.evaluate(alpha_hat, prob)
    gt = backward(theta_b, cache, out["g_alpha"], K, H, s_out)
    theta_n, m_n, v_n = _mlp.adam_update(theta_b, gt, m_b, v_b, t, lr, b1, b2, eps)
    return theta_n, m_n, v_n, alpha_hat, out
