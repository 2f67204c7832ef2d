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

For the option of evaluating the loss on chi_CCO (the paper applies the CCO
after the iterations only), cco_vjp gives the gradient of a real function
through the CCO, in the loss module's convention g_z = dL/dRe z + i dL/dIm z:
the chain rule through eta(|chi|), the two real filters G and their box means
(box_mean_t is the transpose of box_mean).
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


def box_mean_t(x: np.ndarray, r: int) -> np.ndarray:
    """Transpose of box_mean: each pixel collects x / cnt from the windows that contain it."""
    M0, M1 = x.shape
    cnt = np.zeros(x.shape)
    for di in range(-r, r + 1):
        for dj in range(-r, r + 1):
            i0, i1 = max(0, -di), min(M0, M0 - di)
            j0, j1 = max(0, -dj), min(M1, M1 - dj)
            cnt[i0:i1, j0:j1] += 1.0
    y = x / cnt
    out = np.zeros_like(x)
    for di in range(-r, r + 1):
        for dj in range(-r, r + 1):
            i0, i1 = max(0, -di), min(M0, M0 - di)
            j0, j1 = max(0, -dj), min(M1, M1 - dj)
            out[i0 + di:i1 + di, j0 + dj:j1 + dj] += y[i0:i1, j0:j1]
    return out


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


def guided_self_vjp(p: np.ndarray, gG: np.ndarray, r: int = 1, eps: float = 1e-2) -> np.ndarray:
    """dL/dp for a real image p given gG = dL/dG, G = guided_self(p): the steps of
    guided_self taken backwards (mu, var, A, b, then G = mean(A) p + mean(b))."""
    mu = box_mean(p, r)
    var = box_mean(p * p, r) - mu * mu
    A = var / (var + eps)
    g_p = box_mean(A, r) * gG                 # through the factor p of G
    g_A = box_mean_t(gG * p, r)               # through mean(A)
    g_b = box_mean_t(gG, r)                   # through mean(b)
    g_A = g_A - mu * g_b                      # b = (1 - A) mu
    g_mu = (1.0 - A) * g_b
    g_var = g_A * eps / (var + eps) ** 2      # A = var / (var + eps)
    g_mu = g_mu - 2.0 * mu * g_var            # var = mean(p^2) - mu^2
    g_p = g_p + 2.0 * p * box_mean_t(g_var, r) + box_mean_t(g_mu, r)
    return g_p


def cco_vjp(chi: np.ndarray, g_out: np.ndarray, tau=3.0, eta_max=0.1, delta=0.5, r=1, eps_gf=1e-2) -> np.ndarray:
    """Gradient with respect to chi of a real function whose gradient with respect to
    chi_CCO = cco(chi) is g_out."""
    G = guided_self(chi.real, r, eps_gf) + 1j * guided_self(chi.imag, r, eps_gf)
    a = np.abs(chi)
    sg = 1.0 / (1.0 + np.exp(-(a - tau) / delta))
    eta = eta_max * sg
    deta = eta_max * sg * (1.0 - sg) / delta  # d eta / d|chi|
    u = (1.0 + eta) * g_out                   # reaches G
    g = guided_self_vjp(chi.real, u.real, r, eps_gf) + 1j * guided_self_vjp(chi.imag, u.imag, r, eps_gf)
    g = g + eta * g_out                       # the term eta chi, eta held fixed
    # through eta(|chi|): dL = Re(conj(g_out) (G + chi)) deta d|chi|, d|chi| = Re(conj(chi) dchi) / |chi|
    c = np.real(np.conj(g_out) * (G + chi)) * deta / a
    return g + c * chi


def image_error(chi_img: np.ndarray, eps_true: np.ndarray) -> float:
    return float(np.linalg.norm((1.0 + chi_img) - eps_true) / np.linalg.norm(eps_true))
