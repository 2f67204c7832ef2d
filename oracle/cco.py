"""Contrast-compensated operator (Sec. 2.4, Eqs. 10-11) and the image error.

CCO:  chi_CCO = (1 + eta) G(chi | chi) + eta chi,
      eta = eta_max * sigmoid((|chi| - tau) / delta),  tau = 3, eta_max = 0.1,
      delta = 0.5 (Sec. 2.4).  Taken literally: not a convex average.
G is the self-guided filter of He et al. (guide = input), which the paper
cites without parameters.  Readings: box radius r = 1 (3 x 3 window),
regulariser eps_gf = 1e-2, window means normalised by the number of in-grid
pixels at the edges, real and imaginary parts filtered separately:
      mu = mean(p), var = mean(p^2) - mu^2, A = var / (var + eps_gf),
      b = (1 - A) mu,  G = mean(A) p + mean(b).

Relative image error (used in Sec. 4.6, never defined there):
      ||(1 + chi_CCO) - eps_true||_2 / ||eps_true||_2 over the inversion grid.
"""
from __future__ import annotations

import numpy as np


def box_mean(p: np.ndarray, r: int) -> np.ndarray:
    M0, M1 = p.shape
    out = np.zeros_like(p)
    cnt = np.zeros(p.shape)
    for di in range(-r, r + 1):
        for dj in range(-r, r + 1):
            i0, i1 = max(0, -di), min(M0, M0 - di)
            j0, j1 = max(0, -dj), min(M1, M1 - dj)
            out[i0:i1, j0:j1] += p[i0 + di:i1 + di, j0 + dj:j1 + dj]
            cnt[i0:i1, j0:j1] += 1.0
    return out / cnt


def guided_self(p: np.ndarray, r: int = 1, eps: float = 1e-2) -> np.ndarray:
    mu = box_mean(p, r)
    var = box_mean(p * p, r) - mu * mu
    A = var / (var + eps)
    b = (1.0 - A) * mu
    return box_mean(A, r) * p + box_mean(b, r)


def cco(chi: np.ndarray, tau=3.0, eta_max=0.1, delta=0.5, r=1, eps_gf=1e-2) -> np.ndarray:
    G = guided_self(chi.real, r, eps_gf) + 1j * guided_self(chi.imag, r, eps_gf)
    eta = eta_max / (1.0 + np.exp(-(np.abs(chi) - tau) / delta))
    return (1.0 + eta) * G + eta * chi


def image_error(chi_img: np.ndarray, eps_true: np.ndarray) -> float:
    return float(np.linalg.norm((1.0 + chi_img) - eps_true) / np.linalg.norm(eps_true))
