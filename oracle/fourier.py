"""Truncated Fourier basis of the induced currents (Sec. 2.3, Eq. 9).

Kept modes per axis: the K consecutive integer frequencies
k = -floor(K/2), ..., ceil(K/2) - 1.  Odd K is the centred set used by the
workloads; even K = 2 M_F is the paper's own choice of four M_F x M_F blocks
at the corners of the DFT spectrum (M_0 = 4 M_F^2 modes).

Synthesis (F_T^*), unnormalised:
    J[i, j] = sum_{ky, kx} alpha[ky, kx] exp(+2 pi i (ky i + kx j) / M)
Analysis (F_T), forward-normalised so that F_T(F_T^*(alpha)) = alpha:
    alpha[ky, kx] = (1/M^2) sum_{i, j} J[i, j] exp(-2 pi i (ky i + kx j) / M)
The adjoint of synthesis is B^H = M^2 F_T.
alpha is laid out [..., K, K] with ky outer and kx inner, both ascending.
"""
from __future__ import annotations

import numpy as np


def modes(K: int) -> np.ndarray:
    return np.arange(K) - K // 2


def dft_matrix(M: int, K: int) -> np.ndarray:
    """E[i, a] = exp(+2 pi i k_a i / M), [M, K]."""
    i = np.arange(M)[:, None]
    k = modes(K)[None, :]
    return np.exp(2j * np.pi * i * k / M)


def synthesize(alpha: np.ndarray, M: int) -> np.ndarray:
    """J = F_T^*(alpha) for alpha[..., K, K] -> J[..., M, M]."""
    E = dft_matrix(M, alpha.shape[-1])
    return E @ alpha @ E.T


def synth_adjoint(g: np.ndarray, K: int) -> np.ndarray:
    """B^H g for g[..., M, M] -> [..., K, K] (unnormalised forward DFT on the kept modes)."""
    M = g.shape[-1]
    E = dft_matrix(M, K)
    return E.conj().T @ g @ E.conj()


def analyze(J: np.ndarray, K: int) -> np.ndarray:
    """alpha = F_T(J) restricted to the kept modes."""
    M = J.shape[-1]
    return synth_adjoint(J, K) / (M * M)
