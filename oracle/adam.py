"""Adam update on the Fourier coefficients (Sec. 3.3: Adam, learning rate 1e-2).

The paper names only the optimiser and its learning rate; beta1 = 0.9,
beta2 = 0.999, eps = 1e-8 and the bias-corrected form are the usual defaults.
Complex coefficients are optimised as independent (Re, Im) real pairs; the
moment buffers m, v have shape alpha.shape + (2,).  t counts steps from 1.
"""
from __future__ import annotations

import numpy as np


def adam_step(alpha, g, m, v, t, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    gr = np.stack([np.real(g), np.imag(g)], axis=-1)
    m = b1 * m + (1.0 - b1) * gr
    v = b2 * v + (1.0 - b2) * gr * gr
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    step = lr * m_hat / (np.sqrt(v_hat) + eps)
    return alpha - (step[..., 0] + 1j * step[..., 1]), m, v
